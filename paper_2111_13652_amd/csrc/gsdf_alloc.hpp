// Allocation of one 16x16 pixel tile (allocate_blocks): shared by the
// allocation kernel and the combined allocation + normals kernel of the
// frame path.
#pragma once

#include <climits>

#include "gsdf_common.hpp"

namespace gsdf {

constexpr int kAllocSet = 1024;  // LDS set capacity (keys) per tile

// Tile (tu, tv): each pixel's ray band is mapped to block keys, collected in
// the LDS set s_keys (neighbouring pixels share almost all of their
// blocks); then every distinct key is inserted into the global table once
// and marked as touched by this frame.  Every thread of the 256-thread
// work-group must call it (it synchronises); red holds 4 words of LDS.
__device__ inline void allocate_tile(const MapView& M, const float* __restrict__ depth, int W, int H, float zmin,
                                     float zmax, const BandConsts& bc, const double* __restrict__ Twc,
                                     int32_t* status, int tu, int tv, unsigned long long* s_keys,
                                     unsigned long long* red) {
    if (!pose_finite(Twc)) {   // the same pose for every thread: a uniform exit
        if (tu == 0 && tv == 0 && threadIdx.x == 0) raise_status(status, GSDF_EINVAL);
        return;
    }
    for (int i = threadIdx.x; i < kAllocSet; i += blockDim.x) s_keys[i] = kEmptyKey;
    __syncthreads();
    const int u = tu * 16 + (threadIdx.x & 15);
    const int v = tv * 16 + (threadIdx.x >> 4);
    const float D = (u < W && v < H) ? depth[(size_t)v * W + u] : 0.0f;
    if (depth_ok(D, zmin, zmax)) {
        const BandRule br = make_band_rule(Twc, bc.ifx, bc.ify, bc.cxf, bc.cyf, bc.invvs, bc.Tf,
                                           bc.Df, bc.nsamples);
        const float xr = pixel_xr(br, u);
        const float yr = pixel_yr(br, v);
        int pm[3] = {INT_MIN, INT_MIN, INT_MIN};
        int pb[3] = {INT_MIN, INT_MIN, INT_MIN};
        for (int k = 0; k < br.nsamples; ++k) {
            int m[3];
            if (!band_sample(br, xr, yr, D, k, m)) continue;
            if (m[0] == pm[0] && m[1] == pm[1] && m[2] == pm[2]) continue;
            pm[0] = m[0];
            pm[1] = m[1];
            pm[2] = m[2];
            const int bx = block_of(m[0]), by = block_of(m[1]), bz = block_of(m[2]);
            if (bx == pb[0] && by == pb[1] && bz == pb[2]) continue;
            pb[0] = bx;
            pb[1] = by;
            pb[2] = bz;
            if (!block_allowed(M, bx, by, bz)) continue;
            const unsigned long long key = pack_key(bx, by, bz);
            unsigned h = (unsigned)mix64(key) & (kAllocSet - 1);
            bool placed = false;
            for (int probe = 0; probe < kAllocSet; ++probe) {
                const unsigned long long old = atomicCAS(&s_keys[h], kEmptyKey, key);
                if (old == kEmptyKey || old == key) {
                    placed = true;
                    break;
                }
                h = (h + 1) & (kAllocSet - 1);
            }
            if (!placed) {  // set full: go to the global table directly
                int created;
                const int32_t slot = hash_insert(M, bx, by, bz, status, &created);
                if (slot >= 0) mark_touched(M, slot);
            }
        }
    }
    __syncthreads();
    unsigned long long probes = 0;
    for (int i = threadIdx.x; i < kAllocSet; i += blockDim.x) {
        const unsigned long long key = s_keys[i];
        if (key == kEmptyKey) continue;
        int bx, by, bz, created;
        unpack_key(key, &bx, &by, &bz);
        // the inserting thread marks a new block; others mark known slots
        const int32_t slot = hash_insert(M, bx, by, bz, status, &created);
        if (slot >= 0) mark_touched(M, slot);
        ++probes;
    }
    probes = block_sum_u64(probes, red);
    if (threadIdx.x == 0) add_stat(M, kStatAllocPairs, probes);
}

}  // namespace gsdf
