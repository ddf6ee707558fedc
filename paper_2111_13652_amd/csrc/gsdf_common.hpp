// Device-side building blocks shared by the gfx950 kernels of libgsdf:
// map layout, block keys, the hash table, and the binary32 ray-band rule.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/gsdf.h"

namespace gsdf {

constexpr int kBlockEdge = 8;
constexpr int kBlockVoxels = 512;

// ---------------------------------------------------------------------------
// Status bits (1 << -code), OR-ed into the caller's status word.
// ---------------------------------------------------------------------------
__device__ inline void raise_status(int32_t* status, int code) {
    if (status) atomicOr(status, 1 << (-code));
}

// A pose (12 float64, row-major 3x4) whose every entry is finite.  Calls
// given anything else do no work and report GSDF_EINVAL on the device.
__device__ inline bool pose_finite(const double* T) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 12; ++k) ok = ok && isfinite(T[k]);
    return ok;
}

// ---------------------------------------------------------------------------
// Block keys: three 21-bit biased coordinates packed into 63 bits.  The
// all-ones word never encodes a valid key and marks an empty hash slot.
// ---------------------------------------------------------------------------
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int kKeyBias = 1 << 20;
constexpr int kKeyMin = -kKeyBias;          // inclusive
constexpr int kKeyMax = kKeyBias - 2;       // inclusive

__host__ __device__ inline bool key_in_range(int bx, int by, int bz) {
    return bx >= kKeyMin && bx <= kKeyMax && by >= kKeyMin && by <= kKeyMax && bz >= kKeyMin &&
           bz <= kKeyMax;
}

__host__ __device__ inline uint64_t pack_key(int bx, int by, int bz) {
    return ((uint64_t)(uint32_t)(bx + kKeyBias) << 42) | ((uint64_t)(uint32_t)(by + kKeyBias) << 21) |
           (uint64_t)(uint32_t)(bz + kKeyBias);
}

__host__ __device__ inline void unpack_key(uint64_t k, int* bx, int* by, int* bz) {
    const uint64_t m = (1ull << 21) - 1;
    *bx = (int)((k >> 42) & m) - kKeyBias;
    *by = (int)((k >> 21) & m) - kKeyBias;
    *bz = (int)(k & m) - kKeyBias;
}

// 64-bit finaliser (Murmur3 fmix64): scatters neighbouring blocks over the table.
__host__ __device__ inline uint64_t mix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// One hash-table entry, 16 bytes: read with a single dwordx4 load.
struct alignas(16) HashEntry {
    uint64_t key;
    int32_t slot;   // pool slot, or -1 while unassigned / when the pool is full
    int32_t pad;
};

// Voxel index inside a block: Morton order of (lx, ly, lz), so every 2x2x2
// sub-cube (8 voxels) is contiguous.
__host__ __device__ inline int spread3(int x) {  // bits b0 b1 b2 -> positions 0, 3, 6
    return (x & 1) | ((x & 2) << 2) | ((x & 4) << 4);
}
__host__ __device__ inline int morton9(int lx, int ly, int lz) {
    return spread3(lx) | (spread3(ly) << 1) | (spread3(lz) << 2);
}

__host__ __device__ inline void demorton9(int r, int* lx, int* ly, int* lz) {
    int x = 0, y = 0, z = 0;
    for (int b = 0; b < 3; ++b) {
        x |= ((r >> (3 * b)) & 1) << b;
        y |= ((r >> (3 * b + 1)) & 1) << b;
        z |= ((r >> (3 * b + 2)) & 1) << b;
    }
    *lx = x;
    *ly = y;
    *lz = z;
}

// Bytes of one voxel record in map.vox.
__host__ __device__ inline int vox_bytes(int storage) {
    return storage == GSDF_FP32 ? 16 : (storage == GSDF_NOGRAD_FP32 ? 4 : 8);
}

// 16-bit storage formats: bf16 (round to nearest even) and IEEE fp16.
__device__ inline float unpack16(unsigned short s, int storage) {
    if (storage == GSDF_BF16) return __uint_as_float((uint32_t)s << 16);
    __half h;
    *reinterpret_cast<unsigned short*>(&h) = s;
    return __half2float(h);
}

__device__ inline unsigned short pack16(float f, int storage) {
    if (storage == GSDF_BF16) {
        uint32_t u = __float_as_uint(f);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);  // NaN
        u += 0x7fffu + ((u >> 16) & 1u);
        return (unsigned short)(u >> 16);
    }
    __half h = __float2half_rn(f);
    return *reinterpret_cast<unsigned short*>(&h);
}

// Aux buffer layout (offsets in bytes from map.aux).
struct AuxLayout {
    size_t block_keys;   // uint64 per pool slot
    size_t counters;     // 64 int32
    size_t stats;        // 16 uint64 work counters (cumulative since reset)
    size_t touched_flag; // int32 per pool slot (per-frame touched marker)
    size_t total;
};

enum Counter { kNumBlocks = 0 };

// Work counters are striped over kStatStripes addresses (work-group b adds
// into stripe b mod kStatStripes): device-scope atomics on one address
// serialise, so a counter hit by thousands of work-groups must be spread.
constexpr int kStatStripes = 64;

// Work counters, used to state the algorithmic bytes a run moved.
enum Stat {
    kStatUpdates = 0,       // (pixel, voxel) fusion updates applied
    kStatPixelVisits = 1,   // (block, pixel) visits by the fusion gather
    kStatFusedVoxels = 2,   // voxels written by fusion
    kStatFusedBlocks = 3,   // touched blocks processed by fusion
    kStatAllocPairs = 4,    // distinct (tile, block) pairs probed by allocation
    kStatTrackValid = 5,    // valid pixel-iterations in tracking
    kStatTrackUsed = 6,     // pixel-iterations that found an observed voxel
    kStatCount = 16
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline AuxLayout aux_layout(const gsdf_map_desc& d) {
    AuxLayout a;
    size_t nb = (size_t)d.max_blocks;
    size_t o = 0;
    a.block_keys = o;   o = align256(o + nb * 8);
    a.counters = o;     o = align256(o + 64 * 4);
    a.stats = o;        o = align256(o + (size_t)kStatCount * kStatStripes * 8);
    a.touched_flag = o; o = align256(o + nb * 4);
    a.total = o;
    return a;
}

// Device view of a map, passed to kernels by value.
struct MapView {
    HashEntry* hash;
    uint64_t mask;          // hash_slots - 1
    void* vox;
    float* weight;
    uint64_t* block_keys;
    int32_t* counters;
    unsigned long long* stats;
    int32_t* touched_flag;
    int32_t max_blocks;
    int32_t bounded;
    int32_t bmin[3], bmax[3];
    float voxel_size;
    float truncation;
    double voxel_size_d;
    double truncation_d;
};

inline MapView make_view(const gsdf_map& m) {
    MapView v;
    AuxLayout a = aux_layout(m.desc);
    char* aux = (char*)m.aux;
    v.hash = (HashEntry*)m.hash;
    v.mask = (uint64_t)m.desc.hash_slots - 1;
    v.vox = m.vox;
    v.weight = (float*)m.weight;
    v.block_keys = (uint64_t*)(aux + a.block_keys);
    v.counters = (int32_t*)(aux + a.counters);
    v.stats = (unsigned long long*)(aux + a.stats);
    v.touched_flag = (int32_t*)(aux + a.touched_flag);
    v.max_blocks = (int32_t)m.desc.max_blocks;
    v.bounded = m.desc.bounded;
    for (int i = 0; i < 3; ++i) {
        v.bmin[i] = m.desc.bmin[i];
        v.bmax[i] = m.desc.bmax[i];
    }
    v.voxel_size = (float)m.desc.voxel_size;
    v.truncation = (float)m.desc.truncation;
    v.voxel_size_d = m.desc.voxel_size;
    v.truncation_d = m.desc.truncation;
    return v;
}

__device__ inline bool block_allowed(const MapView& M, int bx, int by, int bz) {
    if (!key_in_range(bx, by, bz)) return false;
    if (!M.bounded) return true;
    return bx >= M.bmin[0] && bx < M.bmax[0] && by >= M.bmin[1] && by < M.bmax[1] &&
           bz >= M.bmin[2] && bz < M.bmax[2];
}

// Stored values of voxel vi (pool index slot*512 + morton): returns W and
// sets psi (sum w d / W for the float32 record, psi/T times T for the
// 16-bit pack, both in binary32) and the gradient record g (accumulated
// normals, or their weighted mean).  psi and g are left unset when W <= 0.
__device__ inline float load_voxel(const MapView& M, int storage, int64_t vi, float* psi, float g[3]) {
    const float Wv = M.weight[vi];
    if (!(Wv > 0.0f)) return Wv;
    if (storage == GSDF_FP32) {
        const float4 r = reinterpret_cast<const float4*>(M.vox)[vi];
        *psi = r.x / Wv;
        g[0] = r.y;
        g[1] = r.z;
        g[2] = r.w;
    } else if (storage == GSDF_NOGRAD_FP32) {
        *psi = reinterpret_cast<const float*>(M.vox)[vi] / Wv;
        g[0] = g[1] = g[2] = 0.0f;
    } else {
        const ushort4 r = reinterpret_cast<const ushort4*>(M.vox)[vi];
        *psi = unpack16(r.x, storage) * M.truncation;
        g[0] = unpack16(r.y, storage);
        g[1] = unpack16(r.z, storage);
        g[2] = unpack16(r.w, storage);
    }
    return Wv;
}

// XCD-aware order of work-groups: MI355X dispatches work-groups to its 8
// XCDs in turn (b on XCD b mod 8), each XCD with its own L2.  band_rank(b,
// n) is a permutation of 0 .. n-1 that gives the work-groups of one XCD
// consecutive ranks, so that work-groups that read neighbouring data (the
// same map blocks) share an L2.
constexpr int kXcds = 8;
__device__ inline int band_rank(int b, int n) {
    const int x = b % kXcds;
    int start = 0;
    for (int y = 0; y < x; ++y) start += (n - y + kXcds - 1) / kXcds;   // work-groups on XCD y
    return start + b / kXcds;
}

// Hardware id (0..7) of the XCD the calling wave runs on (register XCC_ID).
__device__ inline unsigned xcc_id() { return (unsigned)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xfu; }

// Pool slot of block (bx,by,bz), or -1.  Linear probing; an empty slot ends
// the search.  Only valid after the kernel that inserted the key finished.
__device__ inline int32_t hash_find(const MapView& M, int bx, int by, int bz) {
    if (!key_in_range(bx, by, bz)) return -1;
    const uint64_t key = pack_key(bx, by, bz);
    uint64_t h = mix64(key) & M.mask;
    for (uint64_t probe = 0; probe <= M.mask; ++probe) {
        const uint4 e = *reinterpret_cast<const uint4*>(&M.hash[h]);
        const uint64_t k = (uint64_t)e.x | ((uint64_t)e.y << 32);
        if (k == key) return (int32_t)e.z;
        if (k == kEmptyKey) return -1;
        h = (h + 1) & M.mask;
    }
    return -1;
}

// Insert a block key if absent.  The winner of the compare-and-swap takes a
// pool slot from the block counter.  Returns the block's pool slot when it
// is known to this thread (-1 while another thread is still assigning it,
// or when the table or pool is full); *created = 1 for the inserting thread.
__device__ inline int32_t hash_insert(const MapView& M, int bx, int by, int bz, int32_t* status,
                                      int* created) {
    *created = 0;
    const uint64_t key = pack_key(bx, by, bz);
    uint64_t h = mix64(key) & M.mask;
    for (uint64_t probe = 0; probe <= M.mask; ++probe) {
        unsigned long long* kp = reinterpret_cast<unsigned long long*>(&M.hash[h].key);
        const uint4 e = *reinterpret_cast<const uint4*>(&M.hash[h]);
        const uint64_t k = (uint64_t)e.x | ((uint64_t)e.y << 32);
        if (k == key) return (int32_t)e.z;
        if (k == kEmptyKey) {
            const uint64_t old = atomicCAS(kp, (unsigned long long)kEmptyKey, (unsigned long long)key);
            if (old == kEmptyKey) {
                const int32_t slot = atomicAdd(&M.counters[kNumBlocks], 1);
                if (slot < M.max_blocks) {
                    M.hash[h].slot = slot;
                    M.block_keys[slot] = key;
                    *created = 1;
                    return slot;
                }
                raise_status(status, GSDF_ECAPACITY);
                return -1;
            }
            if (old == key) return -1;  // inserted concurrently: slot not known yet
        }
        h = (h + 1) & M.mask;
    }
    raise_status(status, GSDF_ECAPACITY);
    return -1;
}

// Sum over the 64 lanes of a wave (every lane gets the total).
__device__ inline unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Record that a block is touched by the current frame: an idempotent flag
// (plain stores; the fusion kernel that consumes it runs later).
__device__ inline void mark_touched(const MapView& M, int32_t slot) {
    if (M.touched_flag[slot] == 0) M.touched_flag[slot] = 1;
}

// Sum over a work-group (every thread passes its value; thread 0 gets the
// total).  `scratch` holds one entry per wave.
__device__ inline unsigned long long block_sum_u64(unsigned long long x, unsigned long long* scratch) {
    x = wave_sum_u64(x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) scratch[wave] = x;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)((blockDim.x + 63) / 64); ++w) t += scratch[w];
    __syncthreads();
    return t;
}

// Add to a work counter (one call per work-group).
__device__ inline void add_stat(const MapView& M, int k, unsigned long long v) {
    if (v) atomicAdd(&M.stats[(size_t)k * kStatStripes + (blockIdx.x & (kStatStripes - 1))], v);
}

// ---------------------------------------------------------------------------
// The ray band of a pixel, decided in binary32 with a fixed operation order
// (no contraction): sample z_k = (D - T) + k (v_s / 2), camera point
// (z xr, z yr, z), world q_i = ((R_i0 X + R_i1 Y) + R_i2 z) + t_i, voxel
// floor(q v_s^-1 + 1/2).  Constants are float32 roundings of the float64
// camera, pose and map parameters.
// ---------------------------------------------------------------------------
struct BandRule {
    float ifx, ify, cxf, cyf, invvs, Tf, Df;
    float R[9], t[3];
    int nsamples;
};

__device__ inline BandRule make_band_rule(const double* T, float ifx, float ify, float cxf,
                                          float cyf, float invvs, float Tf, float Df, int nsamples) {
    BandRule b;
    b.ifx = ifx;
    b.ify = ify;
    b.cxf = cxf;
    b.cyf = cyf;
    b.invvs = invvs;
    b.Tf = Tf;
    b.Df = Df;
    b.nsamples = nsamples;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) b.R[3 * i + j] = (float)T[4 * i + j];
        b.t[i] = (float)T[4 * i + 3];
    }
    return b;
}

// Single-rounding binary32 operations.  HIP's __fmul_rn / __fadd_rn are
// plain operators that the compiler may fuse into FMAs; the decision
// arithmetic below must round after every operation, so contraction is
// switched off in these helpers (HIP honours the pragma).
__device__ inline float mul_rn(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ inline float add_rn(float a, float b) {
#pragma clang fp contract(off)
    return a + b;
}
__device__ inline float sub_rn(float a, float b) {
#pragma clang fp contract(off)
    return a - b;
}

// Voxel coordinate of band sample k of pixel (u, v) with depth D.
// Returns false for samples at or behind the camera (z <= 0).
__device__ inline bool band_sample(const BandRule& b, float xr, float yr, float D, int k, int* m) {
#pragma clang fp contract(off)
    const float z = add_rn(sub_rn(D, b.Tf), mul_rn((float)k, b.Df));
    if (!(z > 0.0f)) return false;
    const float X = mul_rn(z, xr);
    const float Y = mul_rn(z, yr);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float a = mul_rn(b.R[3 * i + 0], X);
        const float c = mul_rn(b.R[3 * i + 1], Y);
        const float e = mul_rn(b.R[3 * i + 2], z);
        const float q = add_rn(add_rn(add_rn(a, c), e), b.t[i]);
        m[i] = (int)floorf(add_rn(mul_rn(q, b.invvs), 0.5f));
    }
    return true;
}

__device__ inline float pixel_xr(const BandRule& b, int u) { return mul_rn(sub_rn((float)u, b.cxf), b.ifx); }
__device__ inline float pixel_yr(const BandRule& b, int v) { return mul_rn(sub_rn((float)v, b.cyf), b.ify); }

// Floor division by 8 (arithmetic shift on two's complement).
__device__ inline int block_of(int m) { return m >> 3; }

__device__ inline bool depth_ok(float D, float zmin, float zmax) {
    return D > 0.0f && D >= zmin && D <= zmax && D <= 3.0e38f;
}

// Host-side float32 constants of the band rule.
struct BandConsts {
    float ifx, ify, cxf, cyf, invvs, Tf, Df;
    int nsamples;
};

inline BandConsts band_consts(const gsdf_camera& c, double voxel_size, double truncation) {
    BandConsts k;
    k.ifx = (float)(1.0 / c.fx);
    k.ify = (float)(1.0 / c.fy);
    k.cxf = (float)c.cx;
    k.cyf = (float)c.cy;
    k.invvs = (float)(1.0 / voxel_size);
    k.Tf = (float)truncation;
    k.Df = (float)(voxel_size / 2.0);
    k.nsamples = (int)std::floor(2.0 * truncation / (voxel_size / 2.0) + 0.5) + 1;
    return k;
}

}  // namespace gsdf
