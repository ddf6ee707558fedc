// Map buffers, block allocation (Sec. 5.3 setup, 8^3 blocks of Sec. 3.1),
// export / import of blocks, status strings and the kernel timer.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <new>
#include <vector>

#include "gsdf_alloc.hpp"
#include "gsdf_common.hpp"
#include "gsdf_host.hpp"

namespace gsdf {

// ---------------------------------------------------------------------------
// Kernel timer: HIP events recorded around the launches of the kernel ids
// selected in a caller-owned gsdf_timer (attached to a map).
// ---------------------------------------------------------------------------
}  // namespace gsdf

struct gsdf_timer {
    std::mutex mu;
    uint32_t mask = 0;  // bit k: time kernel id k
    std::vector<std::pair<hipEvent_t, hipEvent_t>> done[GSDF_K_COUNT];
    hipEvent_t open[GSDF_K_COUNT] = {};
    std::vector<hipEvent_t> pool;
};

namespace gsdf {
namespace {
hipEvent_t take_event(gsdf_timer& t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Return every recorded event to the pool and clear the totals.
void recycle(gsdf_timer& t) {
    for (int k = 0; k < GSDF_K_COUNT; ++k) {
        for (auto& p : t.done[k]) {
            t.pool.push_back(p.first);
            t.pool.push_back(p.second);
        }
        t.done[k].clear();
        if (t.open[k]) {
            t.pool.push_back(t.open[k]);
            t.open[k] = nullptr;
        }
    }
}
}  // namespace

bool timing_on(gsdf_timer* t, int id) { return (t->mask >> id) & 1u; }

void timing_begin(gsdf_timer* t, int id, hipStream_t s) {
    std::lock_guard<std::mutex> g(t->mu);
    hipEvent_t e = take_event(*t);
    if (e && hipEventRecord(e, s) == hipSuccess) t->open[id] = e;
}

void timing_end(gsdf_timer* t, int id, hipStream_t s) {
    std::lock_guard<std::mutex> g(t->mu);
    hipEvent_t b = t->open[id];
    t->open[id] = nullptr;
    if (!b) return;
    hipEvent_t e = take_event(*t);
    if (e && hipEventRecord(e, s) == hipSuccess) t->done[id].push_back({b, e});
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void k_reset_hash(HashEntry* h, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint4 e;
        e.x = 0xffffffffu;
        e.y = 0xffffffffu;
        e.z = 0xffffffffu;  // slot -1
        e.w = 0u;
        *reinterpret_cast<uint4*>(&h[i]) = e;
    }
}

// Zero `n16` 16-byte words.
__global__ void k_zero16(uint4* p, uint64_t n16) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n16; i += (uint64_t)gridDim.x * blockDim.x) p[i] = make_uint4(0, 0, 0, 0);
}

// One work-group per 16x16 pixel tile.  The tile first collects the distinct
// block keys of its pixels' ray bands in an LDS set (neighbouring pixels
// share almost all of their blocks), then inserts each distinct key into
// the global table once and records it as touched by this frame.
__global__ __launch_bounds__(256) void k_allocate(MapView M, const float* __restrict__ depth, int W,
                                                  int H, float zmin, float zmax, BandConsts bc,
                                                  const double* __restrict__ Twc, int32_t* status) {
    __shared__ unsigned long long s_keys[kAllocSet];
    __shared__ unsigned long long red[4];
    allocate_tile(M, depth, W, H, zmin, zmax, bc, Twc, status, blockIdx.x, blockIdx.y, s_keys, red);
}

__global__ void k_sum_stats(MapView M, unsigned long long* out) {
    const int k = threadIdx.x;
    if (k >= kStatCount) return;
    unsigned long long s = 0;
    for (int j = 0; j < kStatStripes; ++j) s += M.stats[(size_t)k * kStatStripes + j];
    out[k] = s;
}

__global__ void k_num_blocks(MapView M, int32_t* n_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int32_t n = M.counters[kNumBlocks];
        n_out[0] = n < M.max_blocks ? n : M.max_blocks;
    }
}

__global__ void k_export_keys(MapView M, int32_t* keys_out, int32_t* n_out) {
    int32_t n = M.counters[kNumBlocks];
    n = n < M.max_blocks ? n : M.max_blocks;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && n_out) n_out[0] = n;
    if (i >= n) return;
    int bx, by, bz;
    unpack_key(M.block_keys[i], &bx, &by, &bz);
    keys_out[3 * i] = bx;
    keys_out[3 * i + 1] = by;
    keys_out[3 * i + 2] = bz;
}

// One thread per voxel: canonical order lx + 8 ly + 64 lz within a block.
__global__ void k_export_voxels(MapView M, int storage, int32_t n_blocks, float* psi_out,
                                float* g_out, float* w_out) {
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= (int64_t)n_blocks * kBlockVoxels) return;
    const int slot = (int)(gi / kBlockVoxels);
    const int c = (int)(gi % kBlockVoxels);
    const int lx = c & 7, ly = (c >> 3) & 7, lz = c >> 6;
    const int64_t vi = (int64_t)slot * kBlockVoxels + morton9(lx, ly, lz);
    const float Wv = M.weight[vi];
    float psi, g0, g1, g2;
    if (storage == GSDF_FP32) {
        const float4 r = reinterpret_cast<const float4*>(M.vox)[vi];
        psi = Wv > 0.0f ? r.x / Wv : 0.0f;
        g0 = r.y;
        g1 = r.z;
        g2 = r.w;
    } else if (storage == GSDF_NOGRAD_FP32) {
        const float r = reinterpret_cast<const float*>(M.vox)[vi];
        psi = Wv > 0.0f ? r / Wv : 0.0f;
        g0 = g1 = g2 = 0.0f;
    } else {
        const ushort4 p = reinterpret_cast<const ushort4*>(M.vox)[vi];
        psi = unpack16(p.x, storage) * M.truncation;
        g0 = unpack16(p.y, storage);
        g1 = unpack16(p.z, storage);
        g2 = unpack16(p.w, storage);
    }
    psi_out[gi] = psi;
    g_out[3 * gi] = g0;
    g_out[3 * gi + 1] = g1;
    g_out[3 * gi + 2] = g2;
    w_out[gi] = Wv;
}

__global__ void k_import_keys(MapView M, const int32_t* keys, int32_t n, int32_t* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int bx = keys[3 * i], by = keys[3 * i + 1], bz = keys[3 * i + 2];
    if (!key_in_range(bx, by, bz)) {
        raise_status(status, GSDF_EINVAL);
        return;
    }
    int created;
    hash_insert(M, bx, by, bz, status, &created);
}

__global__ void k_import_voxels(MapView M, int storage, const int32_t* keys, int32_t n,
                                const float* psi, const float* g, const float* w) {
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= (int64_t)n * kBlockVoxels) return;
    const int i = (int)(gi / kBlockVoxels);
    const int c = (int)(gi % kBlockVoxels);
    const int32_t slot = hash_find(M, keys[3 * i], keys[3 * i + 1], keys[3 * i + 2]);
    if (slot < 0) return;
    const int lx = c & 7, ly = (c >> 3) & 7, lz = c >> 6;
    const int64_t vi = (int64_t)slot * kBlockVoxels + morton9(lx, ly, lz);
    const float Wv = w[gi];
    M.weight[vi] = Wv;
    if (storage == GSDF_FP32) {
        reinterpret_cast<float4*>(M.vox)[vi] =
            make_float4(psi[gi] * Wv, g[3 * gi], g[3 * gi + 1], g[3 * gi + 2]);
    } else if (storage == GSDF_NOGRAD_FP32) {
        reinterpret_cast<float*>(M.vox)[vi] = psi[gi] * Wv;
    } else {
        reinterpret_cast<ushort4*>(M.vox)[vi] =
            make_ushort4(pack16(psi[gi] / M.truncation, storage), pack16(g[3 * gi], storage),
                         pack16(g[3 * gi + 1], storage), pack16(g[3 * gi + 2], storage));
    }
}

}  // namespace gsdf

using namespace gsdf;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int gsdf_map_buffer_sizes(const gsdf_map_desc* desc, size_t sizes_out[4]) {
    if (!desc || !sizes_out || !valid_desc(*desc)) return GSDF_EINVAL;
    const size_t nv = (size_t)desc->max_blocks * kBlockVoxels;
    sizes_out[0] = (size_t)desc->hash_slots * sizeof(HashEntry);
    sizes_out[1] = nv * (size_t)vox_bytes(desc->storage);
    sizes_out[2] = nv * 4;
    sizes_out[3] = aux_layout(*desc).total;
    return GSDF_OK;
}

int gsdf_map_reset(gsdf_map* map, void* stream) {
    if (!valid_map(map)) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    size_t sizes[4];
    gsdf_map_buffer_sizes(&map->desc, sizes);
    const int grid = 2048;
    k_reset_hash<<<grid, 256, 0, s>>>((HashEntry*)map->hash, (uint64_t)map->desc.hash_slots);
    k_zero16<<<grid, 256, 0, s>>>((uint4*)map->vox, sizes[1] / 16);
    k_zero16<<<grid, 256, 0, s>>>((uint4*)map->weight, sizes[2] / 16);
    k_zero16<<<grid, 256, 0, s>>>((uint4*)map->aux, sizes[3] / 16);
    return launch_status();
}

int gsdf_map_num_blocks(const gsdf_map* map, int32_t* n_dev, void* stream) {
    if (!valid_map(map) || !n_dev) return GSDF_EINVAL;
    k_num_blocks<<<1, 64, 0, (hipStream_t)stream>>>(make_view(*map), n_dev);
    return launch_status();
}

int gsdf_allocate_blocks(gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                         const double* T_wc_dev, int32_t* status_dev, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !T_wc_dev) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const BandConsts bc = band_consts(*cam, map->desc.voxel_size, map->desc.truncation);
    dim3 grid(ceil_div(cam->width, 16), ceil_div(cam->height, 16));
    TimedLaunch t(map->timer, GSDF_K_ALLOCATE, s);
    k_allocate<<<grid, 256, 0, s>>>(make_view(*map), depth_dev, cam->width, cam->height,
                                      cam->zmin, cam->zmax, bc, T_wc_dev, status_dev);
    return launch_status();
}

int gsdf_map_counters(const gsdf_map* map, uint64_t* out_dev, void* stream) {
    if (!valid_map(map) || !out_dev) return GSDF_EINVAL;
    k_sum_stats<<<1, 64, 0, (hipStream_t)stream>>>(make_view(*map), (unsigned long long*)out_dev);
    return launch_status();
}

int gsdf_export_keys(const gsdf_map* map, int32_t* keys_out_dev, int32_t* n_dev, void* stream) {
    if (!valid_map(map) || !keys_out_dev) return GSDF_EINVAL;
    const int n = (int)map->desc.max_blocks;
    k_export_keys<<<ceil_div(n, 256), 256, 0, (hipStream_t)stream>>>(make_view(*map), keys_out_dev,
                                                                     n_dev);
    return launch_status();
}

int gsdf_export_voxels(const gsdf_map* map, int32_t n_blocks, float* psi_dev, float* g_dev,
                       float* w_dev, void* stream) {
    if (!valid_map(map) || n_blocks < 0 || n_blocks > map->desc.max_blocks || !psi_dev || !g_dev ||
        !w_dev)
        return GSDF_EINVAL;
    if (n_blocks == 0) return GSDF_OK;
    const int64_t nv = (int64_t)n_blocks * kBlockVoxels;
    k_export_voxels<<<(unsigned)((nv + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        make_view(*map), map->desc.storage, n_blocks, psi_dev, g_dev, w_dev);
    return launch_status();
}

int gsdf_import_blocks(gsdf_map* map, const int32_t* keys_dev, int32_t n, const float* psi_dev,
                       const float* g_dev, const float* w_dev, int32_t* status_dev, void* stream) {
    if (!valid_map(map) || n < 0 || !keys_dev || !psi_dev || !g_dev || !w_dev) return GSDF_EINVAL;
    if (n == 0) return GSDF_OK;
    hipStream_t s = (hipStream_t)stream;
    const MapView M = make_view(*map);
    k_import_keys<<<ceil_div(n, 256), 256, 0, s>>>(M, keys_dev, n, status_dev);
    const int64_t nv = (int64_t)n * kBlockVoxels;
    k_import_voxels<<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(M, map->desc.storage, keys_dev, n,
                                                                psi_dev, g_dev, w_dev);
    return launch_status();
}

int gsdf_timer_create(uint32_t mask, gsdf_timer** out) {
    if (!out) return GSDF_EINVAL;
    gsdf_timer* t = new (std::nothrow) gsdf_timer;
    if (!t) return GSDF_EINVAL;
    t->mask = mask;
    *out = t;
    return GSDF_OK;
}

int gsdf_timer_destroy(gsdf_timer* t) {
    if (!t) return GSDF_OK;
    {
        std::lock_guard<std::mutex> g(t->mu);
        recycle(*t);
        for (hipEvent_t e : t->pool) hipEventDestroy(e);
        t->pool.clear();
    }
    delete t;
    return GSDF_OK;
}

int gsdf_timer_select(gsdf_timer* t, uint32_t mask) {
    if (!t) return GSDF_EINVAL;
    std::lock_guard<std::mutex> g(t->mu);
    recycle(*t);
    t->mask = mask;
    return GSDF_OK;
}

int gsdf_timer_read(gsdf_timer* t, int32_t kernel_id, double* total_ms, int64_t* launches) {
    if (!t || kernel_id < 0 || kernel_id >= GSDF_K_COUNT || !total_ms || !launches) return GSDF_EINVAL;
    std::lock_guard<std::mutex> g(t->mu);
    double sum = 0;
    for (auto& p : t->done[kernel_id]) {
        if (hipEventSynchronize(p.second) != hipSuccess) return GSDF_EHIP;
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess) return GSDF_EHIP;
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)t->done[kernel_id].size();
    return GSDF_OK;
}

const char* gsdf_status_string(int32_t code) {
    switch (code) {
        case GSDF_OK: return "ok";
        case GSDF_EINVAL: return "invalid argument";
        case GSDF_ECAPACITY: return "hash table or block pool full";
        case GSDF_EHIP: return "HIP error";
        case GSDF_ENOTPD: return "Gauss-Newton system not positive definite";
        case GSDF_ELOST: return "tracking lost";
        default: return "unknown status";
    }
}

}  // extern "C"
