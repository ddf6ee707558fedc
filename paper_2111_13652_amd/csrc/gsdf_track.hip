// track_frame: direct SDF tracking with one voxel lookup per pixel
// (Gradient-SDF Sec. 4.1, Eq. (5) and (14)-(16)), Huber-weighted
// Gauss-Newton, and the damped 6x6 Cholesky solve (LDL^T form) with a left SE(3) update
// (Sec. 5.1), all on the device.
//
// A frame is two launches: one kernel builds every pyramid level, and one
// kernel whose work-groups are all resident at once (one per CU) runs every
// Gauss-Newton iteration of every level.  In an iteration each thread walks a strided
// set of pixels and accumulates, in float32 registers, the 21 upper entries
// of H = sum w J J^T, the 6 of b = sum w J r, the energy, the count of
// pixels used and the count of valid pixels.  Four threads' values are
// added once more in float32; from there every sum is float64: LDS across
// the waves of a work-group, then one partial per work-group, then one sum
// per leaf, a leaf being up to 16 work-groups that
// run on one XCD (added by the first work-group of the leaf once every
// partial of the leaf carries the iteration's tag; the partials stay in
// that XCD's L2).  Every work-group then reads the leaf sums the same
// way, adds them in the same fixed order and solves the 6x6 system itself,
// so all of them hold the bit-identical new pose without a round trip
// through a publisher; work-group 0 writes the final pose.
// Waits are bounded spins, so every wave exits even if something went
// wrong.  Float64 partial sums keep the rounding noise of b far below what a
// rank-deficient H (a lone sphere) would amplify through the damping.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gsdf_common.hpp"
#include "gsdf_host.hpp"
#include "gsdf_se3.hpp"

namespace gsdf {

constexpr int kNE = 30;          // 21 H + 6 b + energy + used + valid
constexpr int kPartStride = 32;  // doubles per work-group partial
constexpr int kTrackBlock = 512;
constexpr int kMaxGroups = 2048;
constexpr unsigned kJoinPolls = 1u << 24;   // default bounds of the waits
constexpr unsigned kTagPolls = 1u << 20;

struct TrackLevel {
    const float* depth;
    int W, H;
    double ifx, ify, cx, cy;
};

struct TrackArgs {
    TrackLevel lv[4];
    int levels;
    int iters[4];
    float zmin, zmax, delta;
    double inv_vs, vs;
    double damping;
    float min_inlier_frac;
    unsigned tag_polls;    // bound on the polls of one tagged word
    unsigned join_polls;   // bound on the polls of the level-boundary pose
    unsigned long long* clocks;   // optional per-iteration wall-clock stamps of work-group 0
    int device_scope;      // every partial through device-scope memory (same sums, slower)
};

// Compensated (Kahan) float32 accumulation: after any number of add()s,
// value() is the sum with O(eps) rather than O(n eps) error.
struct Kahan {
    float s = 0.0f, c = 0.0f;
    __device__ inline void add(float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ inline float value() const { return s - c; }
};

// Accumulate the normal equations of the pixels this thread owns at `pose`.
//
// FP32 storage (the plain path): each pixel's world point and its nearest
// voxel are formed in float64, then the offset from the voxel goes to
// float32; sums are float32 per thread.
// 16-bit storage (the precision form): all per-pixel arithmetic is float32,
// camera-relative: q - v_s m_c = R x + t_r with m_c the voxel nearest the
// camera centre and t_r = t - v_s m_c (|t_r| < v_s), so no float32 value
// holds an absolute coordinate at the voxel association; sums are
// compensated (Kahan) float32.  Only the pose itself is float64.
//
// A thread takes its pixels kTrackBatch at a time and issues each stage's
// loads for the whole batch before using any of them (depths, then the
// first hash probe of each, then weight and voxel record together), so a
// batch costs three dependent memory round trips instead of four per
// pixel.  Hash collisions fall back to the probing loop.  The pixels are
// first, first + stride, ... below end.
constexpr int kTrackBatch = 3;

template <int STORAGE>
__device__ inline void accumulate(const MapView& M, const TrackLevel& L, const TrackArgs& a,
                                  const double* pose, int first, int stride, int end, const float* Dpre,
                                  float acc[kNE], float cmp[kNE]) {
    constexpr bool kPrecision = STORAGE == GSDF_BF16 || STORAGE == GSDF_FP16;
    constexpr int B = kTrackBatch;
    Kahan ks[kNE];
#pragma unroll
    for (int k = 0; k < kNE; ++k) acc[k] = 0.0f;
    double R[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) R[3 * i + j] = pose[4 * i + j];
        t[i] = pose[4 * i + 3];
    }
    // camera-relative float32 pose (precision form)
    float Rf[9], trf[3], mcf[3];
    int mc[3];
#pragma unroll
    for (int i = 0; i < 9; ++i) Rf[i] = (float)R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        mc[i] = (int)floor(t[i] * a.inv_vs + 0.5);
        trf[i] = (float)(t[i] - a.vs * (double)mc[i]);
        mcf[i] = (float)(a.vs * (double)mc[i]);
    }
    const float vsf = (float)a.vs, ivsf = (float)a.inv_vs;
    const float ifxf = (float)L.ifx, ifyf = (float)L.ify, cxf = (float)L.cx, cyf = (float)L.cy;

    const int N = end;
    for (int base = first; base < N; base += B * stride) {
        // ---- stage 1: depths (preloaded for the first batch when given)
        float D[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = base + j * stride;
            D[j] = (Dpre && base == first) ? Dpre[j * kTrackBlock + threadIdx.x] : (i < N ? L.depth[i] : 0.0f);
        }
        // ---- stage 2: point, nearest voxel, first hash probe
        int m[B][3];
        float qr[B][3], qf[B][3];
        uint64_t key[B], h[B];
        bool live[B];
        uint4 e[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = base + j * stride;
            live[j] = i < N && depth_ok(D[j], a.zmin, a.zmax);
            if (!live[j]) continue;
            if (kPrecision) ks[29].add(1.0f); else acc[29] += 1.0f;
            const int v = i / L.W;
            const int u = i - v * L.W;
            if (!kPrecision) {
                const double Dd = (double)D[j];
                const double x0 = Dd * (((double)u - L.cx) * L.ifx);
                const double x1 = Dd * (((double)v - L.cy) * L.ify);
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const double q = R[3 * r] * x0 + R[3 * r + 1] * x1 + R[3 * r + 2] * Dd + t[r];
                    m[j][r] = (int)floor(q * a.inv_vs + 0.5);
                    qr[j][r] = (float)(q - a.vs * (double)m[j][r]);
                    qf[j][r] = (float)q;
                }
            } else {
                const float x0 = D[j] * (((float)u - cxf) * ifxf);
                const float x1 = D[j] * (((float)v - cyf) * ifyf);
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const float qc = Rf[3 * r] * x0 + Rf[3 * r + 1] * x1 + Rf[3 * r + 2] * D[j] + trf[r];
                    const int dm = (int)floorf(qc * ivsf + 0.5f);
                    m[j][r] = mc[r] + dm;
                    qr[j][r] = qc - vsf * (float)dm;
                    qf[j][r] = qc + mcf[r];
                }
            }
            const int bx = block_of(m[j][0]), by = block_of(m[j][1]), bz = block_of(m[j][2]);
            if (!key_in_range(bx, by, bz)) {
                live[j] = false;
                continue;
            }
            key[j] = pack_key(bx, by, bz);
            h[j] = mix64(key[j]) & M.mask;
            e[j] = *reinterpret_cast<const uint4*>(&M.hash[h[j]]);
        }
        // ---- stage 3: resolve the probe, then weight and record together
        int64_t vi[B];
        float Wv[B];
        float4 rec32[B];
        ushort4 rec16[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (!live[j]) continue;
            const uint64_t k = (uint64_t)e[j].x | ((uint64_t)e[j].y << 32);
            int32_t slot;
            if (k == key[j]) {
                slot = (int32_t)e[j].z;
            } else if (k == kEmptyKey) {
                slot = -1;
            } else {
                slot = -1;
                uint64_t hh = h[j];
                for (uint64_t probe = 1; probe <= M.mask; ++probe) {
                    hh = (hh + 1) & M.mask;
                    const uint4 f = *reinterpret_cast<const uint4*>(&M.hash[hh]);
                    const uint64_t kk = (uint64_t)f.x | ((uint64_t)f.y << 32);
                    if (kk == key[j]) {
                        slot = (int32_t)f.z;
                        break;
                    }
                    if (kk == kEmptyKey) break;
                }
            }
            if (slot < 0) {
                live[j] = false;
                continue;
            }
            vi[j] = (int64_t)slot * kBlockVoxels + morton9(m[j][0] & 7, m[j][1] & 7, m[j][2] & 7);
            Wv[j] = M.weight[vi[j]];
            if (STORAGE == GSDF_FP32)
                rec32[j] = reinterpret_cast<const float4*>(M.vox)[vi[j]];
            else
                rec16[j] = reinterpret_cast<const ushort4*>(M.vox)[vi[j]];
        }
        // ---- stage 4: residuals and sums.  The three quotients (psi, the
        // normalisation of the gradient, the Huber weight) take the hardware
        // reciprocal and reciprocal square root (1 ulp) instead of the
        // correctly rounded sequences, which are about ten dependent
        // instructions each on every pixel's path.  |g|^2 below the smallest
        // normal float (|g| < 1.1e-19) counts as no gradient.
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (!live[j] || !(Wv[j] > 0.0f)) continue;
            float psi, g0, g1, g2;
            if (STORAGE == GSDF_FP32) {
                psi = rec32[j].x * __builtin_amdgcn_rcpf(Wv[j]);
                g0 = rec32[j].y;
                g1 = rec32[j].z;
                g2 = rec32[j].w;
            } else {
                psi = unpack16(rec16[j].x, STORAGE) * M.truncation;
                g0 = unpack16(rec16[j].y, STORAGE);
                g1 = unpack16(rec16[j].z, STORAGE);
                g2 = unpack16(rec16[j].w, STORAGE);
            }
            const float n2 = g0 * g0 + g1 * g1 + g2 * g2;
            if (!(n2 >= 0x1p-126f)) continue;
            const float inv = __builtin_amdgcn_rsqf(n2);
            const float gh[3] = {g0 * inv, g1 * inv, g2 * inv};
            const float r = psi + gh[0] * qr[j][0] + gh[1] * qr[j][1] + gh[2] * qr[j][2];
            const float J[6] = {gh[0], gh[1], gh[2], qf[j][1] * gh[2] - qf[j][2] * gh[1],
                                qf[j][2] * gh[0] - qf[j][0] * gh[2], qf[j][0] * gh[1] - qf[j][1] * gh[0]};
            const float ar = fabsf(r);
            const float w = ar <= a.delta ? 1.0f : a.delta * __builtin_amdgcn_rcpf(ar);
            const float en = ar <= a.delta ? 0.5f * r * r : a.delta * (ar - 0.5f * a.delta);
            int k = 0;
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const float wj = w * J[p];
#pragma unroll
                for (int q2 = p; q2 < 6; ++q2) {
                    if (kPrecision) ks[k].add(wj * J[q2]); else acc[k] += wj * J[q2];
                    ++k;
                }
            }
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                if (kPrecision) ks[21 + p].add(w * J[p] * r); else acc[21 + p] += w * J[p] * r;
            }
            if (kPrecision) {
                ks[27].add(en);
                ks[28].add(1.0f);
            } else {
                acc[27] += en;
                acc[28] += 1.0f;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kNE; ++k) {
        if (kPrecision) {
            acc[k] = ks[k].s;
            cmp[k] = ks[k].c;
        } else {
            cmp[k] = 0.0f;
        }
    }
}

// Tri-linear residual model (Sec. 4.1 Eq. (12)-(13)): the direct SDF
// tracking the paper compares its single-lookup Taylor model against.  Each
// pixel reads the eight voxels around its point q (cell b = floor(q / v_s),
// corners b + {0, 1}^3, through the hash table when a corner lies in a
// neighbouring block); the distance is the tri-linear interpolant of their
// values and the gradient its derivative (corner differences along each
// axis, weighted bilinearly in the other two).  A pixel is used when all
// eight voxels are observed.  Point and cell in float64, the rest as in the
// Taylor model; the sums use the same layout.
template <int STORAGE>
__device__ inline void accumulate_trilinear(const MapView& M, const TrackLevel& L, const TrackArgs& a,
                                            const double* pose, int first, int stride, int end,
                                            const float* Dpre, float acc[kNE], float cmp[kNE]) {
    constexpr bool kPrecision = STORAGE == GSDF_BF16 || STORAGE == GSDF_FP16;
    constexpr int B = kTrackBatch;
    Kahan ks[kNE];
#pragma unroll
    for (int k = 0; k < kNE; ++k) acc[k] = 0.0f;
    double R[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) R[3 * i + j] = pose[4 * i + j];
        t[i] = pose[4 * i + 3];
    }
    const float ivsf = (float)a.inv_vs;
    const int N = end;
    for (int base = first; base < N; base += B * stride) {
        float D[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = base + j * stride;
            D[j] = (Dpre && base == first) ? Dpre[j * kTrackBlock + threadIdx.x] : (i < N ? L.depth[i] : 0.0f);
        }
        // point, cell, the cell's block
        int cb[B][3];
        float f[B][3], qf[B][3];
        bool live[B];
        int32_t slot0[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = base + j * stride;
            live[j] = i < N && depth_ok(D[j], a.zmin, a.zmax);
            if (!live[j]) continue;
            if (kPrecision) ks[29].add(1.0f); else acc[29] += 1.0f;
            const int v = i / L.W;
            const int u = i - v * L.W;
            const double Dd = (double)D[j];
            const double x0 = Dd * (((double)u - L.cx) * L.ifx);
            const double x1 = Dd * (((double)v - L.cy) * L.ify);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double q = R[3 * r] * x0 + R[3 * r + 1] * x1 + R[3 * r + 2] * Dd + t[r];
                const double sq = q * a.inv_vs;
                cb[j][r] = (int)floor(sq);
                f[j][r] = (float)(sq - (double)cb[j][r]);
                qf[j][r] = (float)q;
            }
            slot0[j] = hash_find(M, block_of(cb[j][0]), block_of(cb[j][1]), block_of(cb[j][2]));
            if (slot0[j] < 0) live[j] = false;
        }
        // the eight corners: weight and stored distance term
        float cw[B][8];
        uint32_t craw[B][8];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (!live[j]) continue;
            const int b0x = block_of(cb[j][0]), b0y = block_of(cb[j][1]), b0z = block_of(cb[j][2]);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int mx = cb[j][0] + (c & 1), my = cb[j][1] + ((c >> 1) & 1), mz = cb[j][2] + (c >> 2);
                const int bx = block_of(mx), by = block_of(my), bz = block_of(mz);
                const int32_t slot =
                    (bx == b0x && by == b0y && bz == b0z) ? slot0[j] : hash_find(M, bx, by, bz);
                if (slot < 0) {
                    cw[j][c] = 0.0f;
                    craw[j][c] = 0u;
                    continue;
                }
                const int64_t vi = (int64_t)slot * kBlockVoxels + morton9(mx & 7, my & 7, mz & 7);
                cw[j][c] = M.weight[vi];
                if (STORAGE == GSDF_FP32)
                    craw[j][c] = __float_as_uint(reinterpret_cast<const float*>(M.vox)[4 * vi]);
                else if (STORAGE == GSDF_NOGRAD_FP32)
                    craw[j][c] = __float_as_uint(reinterpret_cast<const float*>(M.vox)[vi]);
                else
                    craw[j][c] = reinterpret_cast<const unsigned short*>(M.vox)[4 * vi];
            }
        }
        // interpolant, residual, sums
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (!live[j]) continue;
            bool all = true;
            float c[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                all = all && cw[j][k] > 0.0f;
                // the Taylor model's hardware reciprocal (a corner with W = 0
                // gives inf or NaN here and is dropped below)
                c[k] = (STORAGE == GSDF_FP32 || STORAGE == GSDF_NOGRAD_FP32)
                           ? __uint_as_float(craw[j][k]) * __builtin_amdgcn_rcpf(cw[j][k])
                           : unpack16((unsigned short)craw[j][k], STORAGE) * M.truncation;
            }
            if (!all) continue;
            const float wx[2] = {1.0f - f[j][0], f[j][0]};
            const float wy[2] = {1.0f - f[j][1], f[j][1]};
            const float wz[2] = {1.0f - f[j][2], f[j][2]};
            float d = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) d += c[k] * wx[k & 1] * wy[(k >> 1) & 1] * wz[k >> 2];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // k enumerates the other two axes' corner bits
                gx += (c[2 * k + 1] - c[2 * k]) * wy[k & 1] * wz[k >> 1];
                gy += (c[(k & 1) + 4 * (k >> 1) + 2] - c[(k & 1) + 4 * (k >> 1)]) * wx[k & 1] * wz[k >> 1];
                gz += (c[k + 4] - c[k]) * wx[k & 1] * wy[k >> 1];
            }
            const float g[3] = {gx * ivsf, gy * ivsf, gz * ivsf};
            const float r = d;
            const float J[6] = {g[0], g[1], g[2], qf[j][1] * g[2] - qf[j][2] * g[1],
                                qf[j][2] * g[0] - qf[j][0] * g[2], qf[j][0] * g[1] - qf[j][1] * g[0]};
            const float ar = fabsf(r);
            const float w = ar <= a.delta ? 1.0f : a.delta * __builtin_amdgcn_rcpf(ar);
            const float en = ar <= a.delta ? 0.5f * r * r : a.delta * (ar - 0.5f * a.delta);
            int k = 0;
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const float wj = w * J[p];
#pragma unroll
                for (int q2 = p; q2 < 6; ++q2) {
                    if (kPrecision) ks[k].add(wj * J[q2]); else acc[k] += wj * J[q2];
                    ++k;
                }
            }
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                if (kPrecision) ks[21 + p].add(w * J[p] * r); else acc[21 + p] += w * J[p] * r;
            }
            if (kPrecision) {
                ks[27].add(en);
                ks[28].add(1.0f);
            } else {
                acc[27] += en;
                acc[28] += 1.0f;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kNE; ++k) {
        if (kPrecision) {
            acc[k] = ks[k].s;
            cmp[k] = ks[k].c;
        } else {
            cmp[k] = 0.0f;
        }
    }
}

// Work-group sum: every thread writes its kNE sums to LDS (one transpose),
// then 8 threads per entry add kRedChunk values each with independent LDS
// reads, and the first kNE threads combine the 8 parts and store the
// work-group partial with device-scope stores.  (Cross-lane shuffles of
// doubles would chain ~180 dependent LDS permutes per wave.)  Each entry's
// row is 8 chunks of kRedChunk values, kRedPad floats apart, so that the 8
// lanes of one 16-byte read pass (the 8 chunks of an entry) fall in
// different banks.  The plain path adds each chunk (one wave's values) four
// at a time in float32, then those sums and the 8 chunk sums by pairwise
// trees in float64: the serial float64 chain it replaces (64 conversions
// and adds per thread, then 8 more adds) was the longest dependent sequence
// of the sum (measured: 3.5 us less per tracking launch at 640x480).  A
// float32 tree over a whole chunk is 0.6 us faster still but loses what
// float64 keeps: where a thread holds a single pixel its sums are exact
// products, and on an ill-conditioned system (a sphere, whose rotations
// about its centre leave the residuals unchanged) the tracked centre moved
// 40 times further from the float64 oracle's.  The precision form
// (COMP) uses compensated float32 at every stage.  The storing threads are
// lanes of wave 0, so thread 0 (which takes the arrival ticket, where there
// is one) waits for their completion before signalling.
constexpr int kRedChunk = kTrackBlock / 8;
constexpr int kRedPad = kRedChunk + 4;
struct ReduceLds {
    float v[kNE][8 * kRedPad];
    double part[kNE][8];
    double tot[kNE];
};
__device__ inline int red_slot(int t) { return (t / kRedChunk) * kRedPad + t % kRedChunk; }

// Partials and leaf sums of the tracking kernel carry the iteration they
// belong to: the low 16 bits of each float64 word (a relative change below
// 2^-36, the same for every reader) hold the tag, so a reader that sees the
// tag has the value, with no separate signal to wait for first.  Tags are
// 1 + the iteration index (at most 4000 iterations a frame), and the words
// are cleared before each frame.
constexpr unsigned long long kTagMask = 0xffffull;
__device__ inline unsigned long long tag_word(double v, unsigned long long tag) {
    return ((unsigned long long)__double_as_longlong(v) & ~kTagMask) | tag;
}
__device__ inline double untag_word(unsigned long long w) { return __longlong_as_double((long long)(w & ~kTagMask)); }

// A tagged partial (tag != 0) is stored at work-group scope when `local`
// (its reader runs on the same XCD), else at device scope.
template <bool COMP>
__device__ inline void store_partial(const float acc[kNE], const float cmp[kNE], double* partial,
                                     ReduceLds& r, unsigned long long tag = 0, bool local = false) {
    const int slot = red_slot(threadIdx.x);
#pragma unroll
    for (int k = 0; k < kNE; ++k) r.v[k][slot] = COMP ? acc[k] - cmp[k] : acc[k];
    __syncthreads();
    if (threadIdx.x < kNE * 8) {
        const int k = threadIdx.x >> 3, p = threadIdx.x & 7;
        const float4* src = reinterpret_cast<const float4*>(&r.v[k][p * kRedPad]);
        float4 q[kRedChunk / 4];
#pragma unroll
        for (int j = 0; j < kRedChunk / 4; ++j) q[j] = src[j];
        if (COMP) {
            Kahan ks;
#pragma unroll
            for (int j = 0; j < kRedChunk / 4; ++j) {
                ks.add(q[j].x);
                ks.add(q[j].y);
                ks.add(q[j].z);
                ks.add(q[j].w);
            }
            r.part[k][p] = (double)ks.value();
        } else {
            double t[kRedChunk / 4];
#pragma unroll
            for (int j = 0; j < kRedChunk / 4; ++j) t[j] = (double)((q[j].x + q[j].y) + (q[j].z + q[j].w));
#pragma unroll
            for (int w = kRedChunk / 8; w >= 1; w /= 2) {
#pragma unroll
                for (int j = 0; j < w; ++j) t[j] = t[j] + t[j + w];
            }
            r.part[k][p] = t[0];
        }
    }
    __syncthreads();
    if (threadIdx.x < kNE) {
        double s = 0.0;
        if (COMP) {
            Kahan ks;
#pragma unroll
            for (int p = 0; p < 8; ++p) ks.add((float)r.part[threadIdx.x][p]);
            s = (double)ks.value();
        } else {
            double t[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) t[p] = r.part[threadIdx.x][p];
#pragma unroll
            for (int w = 4; w >= 1; w /= 2) {
#pragma unroll
                for (int j = 0; j < w; ++j) t[j] = t[j] + t[j + w];
            }
            s = t[0];
        }
        if (tag && local)
            __hip_atomic_store(reinterpret_cast<unsigned long long*>(&partial[threadIdx.x]), tag_word(s, tag),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else if (tag)
            __hip_atomic_store(reinterpret_cast<unsigned long long*>(&partial[threadIdx.x]), tag_word(s, tag),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_store(&partial[threadIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Sum of `groups` partials (device-scope loads, issued after the signal
// that every one of them was stored).  Thread (k, p) adds entry k of the
// partials p, p+8, ... in that order, with up to sixteen loads in flight.  Result in ne[] of
// thread 0.
template <bool COMP>
__device__ inline void total_partials(const double* partials, int groups, double ne[kNE], ReduceLds& r) {
    if (threadIdx.x < kNE * 8) {
        const int k = threadIdx.x >> 3, p = threadIdx.x & 7;
        double s = 0.0;
        Kahan ks;
        int b = p;
        for (; b + 120 < groups; b += 128) {
            double x[16];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                x[j] = __hip_atomic_load(&partials[(size_t)(b + 8 * j) * kPartStride + k], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (COMP) ks.add((float)x[j]); else s += x[j];
            }
        }
        for (; b + 56 < groups; b += 64) {
            double x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                x[j] = __hip_atomic_load(&partials[(size_t)(b + 8 * j) * kPartStride + k], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (COMP) ks.add((float)x[j]); else s += x[j];
            }
        }
        for (; b < groups; b += 8) {
            const double x = __hip_atomic_load(&partials[(size_t)b * kPartStride + k], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
            if (COMP) ks.add((float)x); else s += x;
        }
        r.part[k][p] = COMP ? (double)ks.value() : s;
    }
    __syncthreads();
    if (threadIdx.x < kNE) {
        const int k = threadIdx.x;
        if (COMP) {
            Kahan ks;
            for (int p = 0; p < 8; ++p) ks.add((float)r.part[k][p]);
            r.tot[k] = (double)ks.value();
        } else {
            double t = 0.0;
            for (int p = 0; p < 8; ++p) t += r.part[k][p];
            r.tot[k] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < kNE; ++k) ne[k] = r.tot[k];
}

// The damped 6x6 solve and the left pose update, by one wave.
//
// Lane i < 6 holds row i of [H + mu I | -b] (mu = damping tr(H)/6).
// Gaussian elimination without pivoting: H + mu I is symmetric positive
// definite, so every pivot is positive and this is its LDL^T factorisation
// (the same solution as a Cholesky solve, with no square roots).  The pivot
// row is broadcast with readlane, each lane below it eliminates its own
// entry, and back substitution broadcasts each unknown as it is found.  Then
// lane k < 12 forms entry k = 4 i + j of exp(x^) T from row i of R and V
// (the closed forms of se3_exp) and column j of T.  ne is the float64 sum
// (21 upper entries of H row by row, then b) in LDS; pose is the 3x4 pose in
// LDS, replaced in place.  Every lane returns the same flag: false when a
// pivot is not positive, with the pose unchanged.

__device__ inline double bcast_lane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __hiloint2double(hi, lo);
}

// 1/p to within an ulp: hardware reciprocal and one Newton step.
__device__ inline double recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    const double e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

__device__ inline int upper_index(int i, int j) { return i * 6 - (i * (i - 1)) / 2 + (j - i); }  // i <= j

__device__ inline bool solve_update_wave(const double* ne, double damping, double* pose) {
    const int lane = threadIdx.x & 63;
    const int i = lane < 6 ? lane : 5;  // lanes 6.. shadow row 5; their values are never read
    double tr = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) tr += ne[upper_index(d, d)];
    const double mu = damping * tr * (1.0 / 6.0);
    double row[7];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double h = ne[i <= c ? upper_index(i, c) : upper_index(c, i)];
        row[c] = c == i ? h + mu : h;
    }
    row[6] = -ne[21 + i];
    double inv_piv[6];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double pr[7];
#pragma unroll
        for (int c = j; c < 7; ++c) pr[c] = bcast_lane(row[c], j);
        ok = ok && pr[j] > 0.0;
        inv_piv[j] = recip(pr[j]);
        const double f = lane > j ? row[j] * inv_piv[j] : 0.0;
#pragma unroll
        for (int c = j + 1; c < 7; ++c) row[c] = fma(-f, pr[c], row[c]);
    }
    if (!ok) return false;
    double x[6];
    double rhs = row[6];
#pragma unroll
    for (int c = 5; c >= 0; --c) {
        x[c] = bcast_lane(rhs * inv_piv[c], c);
        rhs = fma(-row[c], x[c], rhs);
    }
    // exp of the twist (rho, phi) = (x[0..2], x[3..5]); coefficients as in se3_exp
    const double p0 = x[3], p1 = x[4], p2 = x[5];
    const double th2 = p0 * p0 + p1 * p1 + p2 * p2;
    double A, B, C;
    if (th2 < 0.02 * 0.02) {
        // the series of se3_exp in Horner form with reciprocal constants
        // (a division by a constant is a ten-instruction sequence in float64)
        constexpr double a1 = -1.0 / 6.0, a2 = 1.0 / 120.0, a3 = -1.0 / 5040.0, a4 = 1.0 / 362880.0;
        constexpr double b1 = -1.0 / 24.0, b2 = 1.0 / 720.0, b3 = -1.0 / 40320.0, b4 = 1.0 / 3628800.0;
        constexpr double c0 = 1.0 / 6.0, c1 = -1.0 / 120.0, c2 = 1.0 / 5040.0, c3 = -1.0 / 362880.0,
                         c4 = 1.0 / 39916800.0;
        A = 1.0 + th2 * (a1 + th2 * (a2 + th2 * (a3 + th2 * a4)));
        B = 0.5 + th2 * (b1 + th2 * (b2 + th2 * (b3 + th2 * b4)));
        C = c0 + th2 * (c1 + th2 * (c2 + th2 * (c3 + th2 * c4)));
    } else {
        const double th = sqrt(th2);
        const double sn = sin(th), cs = cos(th);
        A = sn / th;
        B = (1.0 - cs) / th2;
        C = (th - sn) / (th2 * th);
    }
    if (lane < 12) {
        const int r = lane >> 2, col = lane & 3;
        // row r of K = phi^ and of K^2 = phi phi^T - th2 I
        const double pr_ = r == 0 ? p0 : (r == 1 ? p1 : p2);
        const double k0 = r == 0 ? 0.0 : (r == 1 ? p2 : -p1);
        const double k1 = r == 0 ? -p2 : (r == 1 ? 0.0 : p0);
        const double k2 = r == 0 ? p1 : (r == 1 ? -p0 : 0.0);
        const double q0 = pr_ * p0 - (r == 0 ? th2 : 0.0);
        const double q1 = pr_ * p1 - (r == 1 ? th2 : 0.0);
        const double q2 = pr_ * p2 - (r == 2 ? th2 : 0.0);
        const double R0 = (r == 0 ? 1.0 : 0.0) + A * k0 + B * q0;
        const double R1 = (r == 1 ? 1.0 : 0.0) + A * k1 + B * q1;
        const double R2 = (r == 2 ? 1.0 : 0.0) + A * k2 + B * q2;
        double out = R0 * pose[col] + R1 * pose[4 + col] + R2 * pose[8 + col];
        if (col == 3) {
            const double V0 = (r == 0 ? 1.0 : 0.0) + B * k0 + C * q0;
            const double V1 = (r == 1 ? 1.0 : 0.0) + B * k1 + C * q1;
            const double V2 = (r == 2 ? 1.0 : 0.0) + B * k2 + C * q2;
            out += V0 * x[0] + V1 * x[1] + V2 * x[2];
        }
        // every lane's reads of the pose above precede this store (the store
        // depends on them, and the wave issues LDS operations in order)
        pose[lane] = out;
    }
    return true;
}

// Memory ordering between work-groups.  Everything one work-group hands to
// another (partial sums, leaf sums, the published pose, tickets and flags) is
// read only with device-scope atomic loads, and written with device-scope
// atomic stores, which the hardware keeps coherent per location across the
// XCDs without cache maintenance: such a store writes through the writer's
// L2, such a load does not return a line its L2 holds clean.  One exception
// keeps a hop inside an XCD: the tracking kernel's partials go to their
// leaf's first work-group, which runs on the same XCD, and are stored at
// work-group scope.  That store leaves the line dirty in the XCD's L2, and
// a device-scope load from the same XCD returns a dirty line of its own L2
// (measured on MI355X: a store-to-load round trip of 0.46 us between two
// work-groups on one XCD against 0.85 us with device-scope stores, and
// 1.2 us between XCDs).  A work-group that does not find itself on its leaf
// leader's XCD (the leader publishes its hardware XCC id) stores its
// partials at device scope instead, so the exchange never depends on the
// dispatch order for its correctness.  A tagged word (the tracking kernel's
// partials and leaf sums) needs nothing more: it is written by one 64-bit
// store, so a reader that sees its tag sees its value.  Elsewhere ordering is all that is
// needed: a producer waits until its device-scope stores have completed
// before it signals (s_waitcnt on all counters, below), and a consumer
// issues its loads only after the signal's value has returned.  A
// release/acquire fence at device scope would add an
// L2 write-back and invalidation per work-group and iteration (measured at
// about 10 % of the kernel at 640x480) to order plain memory operations,
// which this kernel does not exchange.
__device__ inline void complete_device_stores() { __builtin_amdgcn_s_waitcnt(0); }

// Reduction across work-groups: a two-level tree.  Single-launch
// reductions (the normal equations) take kLeaf consecutive work-groups to a
// leaf and use arrival tickets (device-scope atomics on one address
// serialise, so a single ticket for hundreds of work-groups would cost tens
// of microseconds): the last work-group of a leaf adds the leaf's
// partials, the last leaf adds the leaf sums.  The tracking kernel uses no
// tickets and leaves of up to kXcdLeaf work-groups of one XCD: work-group b
// runs on XCD x = b mod 8 (the dispatcher deals work-groups to the XCDs in
// turn) as the i-th (i = b / 8) of that XCD; its partial goes to slot
// x * kPerXcd + i, it belongs to leaf (i / kXcdLeaf) * 8 + x, and the
// member with i mod kXcdLeaf = 0 leads the leaf.  A leaf's partials are
// consecutive, and the leaves of a level are numbered 0 .. nleaf-1 without
// gaps.  Partials and leaf sums are tagged with their iteration (below),
// the leader polls its leaf's partials, and every member polls the leaf
// sums.  Sync words: the tickets, the iteration count of the pose published
// at level boundaries for work-groups that join, an abort flag, and each
// tracking leaf leader's XCC id.  The pyramid
// kernel clears them and the tagged words before each tracking launch.
constexpr int kLeaf = 16;
constexpr int kMaxLeaves = kMaxGroups / kLeaf;
constexpr int kPerXcd = kMaxGroups / kXcds;
// Work-groups per tracking leaf.  Measured on MI355X (one work-group per CU,
// 32 per XCD): 16 beats 32 and 8 by 2.3 us per launch at 640x480 and by
// 5.3-6 us at 1280x720.
constexpr int kXcdLeaf = 16;
static_assert((kMaxGroups / kXcdLeaf) <= kMaxLeaves, "tracking leaves must fit the leaf sums");
__device__ inline int xcd_leaf(int b) { return (b / kXcds / kXcdLeaf) * kXcds + b % kXcds; }
__device__ inline bool xcd_leader(int b) { return (b / kXcds) % kXcdLeaf == 0; }
// leaves of a level with n members (consecutive numbers from 0)
__device__ inline int xcd_leaves(int n) {
    constexpr int span = kXcds * kXcdLeaf;
    return kXcds * (n / span) + min(kXcds, n % span);
}
// one set of partials: a partial per work-group, then one per leaf
constexpr size_t kPartsPerSet = (size_t)(kMaxGroups + kMaxLeaves) * kPartStride;
// Leaf tickets are kTicketStride words (256 B) apart: device-scope atomics
// on one cache line share the memory-side atomic unit.
constexpr int kTicketStride = 64;
enum {
    kSyncLeaf = 0,                                          // [2][kMaxLeaves] x kTicketStride
    kSyncRoot = kSyncLeaf + 2 * kMaxLeaves * kTicketStride,  // [2]
    kSyncPub = kSyncRoot + 2,                               // iterations reflected by the published pose
    kSyncAbort = kSyncPub + 1,
    kSyncXcc = kSyncAbort + 1,                              // [kMaxLeaves] 1 + XCC id of each tracking leaf leader
    kSyncWords = kSyncXcc + kMaxLeaves
};

// Arrival, thread 0 only.  leaf_arrive: true for the last of the kLeaf
// work-groups sharing a leaf ticket; root_arrive: true for the last leaf.
// Before each ticket the work-group's device-scope partial stores have
// completed; the winner reads the others' partials with device-scope loads.
__device__ inline bool leaf_arrive(unsigned* sync, int par, int groups) {
    const int leaf = blockIdx.x / kLeaf;
    const int leaf_size = min(kLeaf, groups - leaf * kLeaf);
    complete_device_stores();
    unsigned* lc = &sync[kSyncLeaf + (par * kMaxLeaves + leaf) * kTicketStride];
    if (__hip_atomic_fetch_add(lc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (unsigned)leaf_size - 1)
        return false;
    __hip_atomic_store(lc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Single-level arrival (grids of at most kSingleLevel work-groups): the
// serialised same-address atomics cost less than a second tree level.
constexpr int kSingleLevel = 16;
__device__ inline bool root_arrive_direct(unsigned* sync, int par, int groups) {
    complete_device_stores();
    unsigned* rc = &sync[kSyncRoot + par];
    if (__hip_atomic_fetch_add(rc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (unsigned)groups - 1)
        return false;
    __hip_atomic_store(rc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

__device__ inline bool root_arrive(unsigned* sync, int par, int groups) {
    const int nleaf = (groups + kLeaf - 1) / kLeaf;
    complete_device_stores();
    unsigned* rc = &sync[kSyncRoot + par];
    if (__hip_atomic_fetch_add(rc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (unsigned)nleaf - 1)
        return false;
    __hip_atomic_store(rc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Two-level sum of the work-group partials: the last work-group of each
// leaf adds the leaf's partials and stores a leaf partial; the last leaf adds
// those.  Returns true (in every thread) for the work-group that holds the
// total, in ne[] of thread 0.  `part` has one partial per work-group,
// `leafpart` one per leaf.
template <bool COMP>
__device__ inline bool reduce_tree(const float acc[kNE], const float cmp[kNE], double* part, double* leafpart,
                                   unsigned* sync, int par, int groups, double ne[kNE], ReduceLds& r,
                                   int* s_flag) {
    store_partial<COMP>(acc, cmp, part + (size_t)blockIdx.x * kPartStride, r);
    if (groups <= kSingleLevel) {
        // few work-groups: one arrival counter, the last sums every partial
        if (threadIdx.x == 0) *s_flag = root_arrive_direct(sync, par, groups) ? 1 : 0;
        __syncthreads();
        if (!*s_flag) return false;
        total_partials<COMP>(part, groups, ne, r);
        return true;
    }
    if (threadIdx.x == 0) *s_flag = leaf_arrive(sync, par, groups) ? 1 : 0;
    __syncthreads();
    if (!*s_flag) return false;
    const int leaf = blockIdx.x / kLeaf;
    const int leaf_size = min(kLeaf, groups - leaf * kLeaf);
    double lsum[kNE];
    total_partials<COMP>(part + (size_t)leaf * kLeaf * kPartStride, leaf_size, lsum, r);
    if (threadIdx.x == 0) {
        for (int k = 0; k < kNE; ++k)
            __hip_atomic_store(&leafpart[(size_t)leaf * kPartStride + k], lsum[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = root_arrive(sync, par, groups) ? 1 : 0;
    }
    __syncthreads();
    if (!*s_flag) return false;
    total_partials<COMP>(leafpart, (groups + kLeaf - 1) / kLeaf, ne, r);
    return true;
}

// The sum of n tagged partials (consecutive, kPartStride apart) of the
// iteration tagged `tag`, in the order of total_partials (thread (k, p) adds
// entry k of the partials p, p+8, ...), each word polled until it carries
// the tag.  Result in r.tot; false (in every thread) on timeout or when
// another work-group aborted.
template <bool COMP>
__device__ inline bool total_leaves(const double* leafpart, int nleaf, unsigned long long tag, const unsigned* sync,
                                    unsigned max_polls, ReduceLds& r) {
    bool ok = true;
    if (threadIdx.x < kNE * 8) {
        const int k = threadIdx.x >> 3, p = threadIdx.x & 7;
        double s = 0.0;
        Kahan ks;
        for (int b0 = p; b0 < nleaf && ok; b0 += 16) {
            const int b1 = b0 + 8;
            const unsigned long long* w0 =
                reinterpret_cast<const unsigned long long*>(&leafpart[(size_t)b0 * kPartStride + k]);
            const unsigned long long* w1 =
                reinterpret_cast<const unsigned long long*>(&leafpart[(size_t)(b1 < nleaf ? b1 : b0) * kPartStride + k]);
            unsigned long long x0 = __hip_atomic_load(w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long x1 =
                b1 < nleaf ? __hip_atomic_load(w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : tag;
            unsigned spins = 0;
            while ((x0 & kTagMask) != tag || (x1 & kTagMask) != tag) {
                if (++spins > max_polls ||
                    ((spins & 255u) == 0u &&
                     __hip_atomic_load(&sync[kSyncAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if ((x0 & kTagMask) != tag) x0 = __hip_atomic_load(w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((x1 & kTagMask) != tag) x1 = __hip_atomic_load(w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (COMP) {
                ks.add((float)untag_word(x0));
                if (b1 < nleaf) ks.add((float)untag_word(x1));
            } else {
                s += untag_word(x0);
                if (b1 < nleaf) s += untag_word(x1);
            }
        }
        r.part[k][p] = COMP ? (double)ks.value() : s;
    }
    if (__syncthreads_or(ok ? 0 : 1)) return false;
    if (threadIdx.x < kNE) {
        const int k = threadIdx.x;
        if (COMP) {
            Kahan ks;
            for (int p = 0; p < 8; ++p) ks.add((float)r.part[k][p]);
            r.tot[k] = (double)ks.value();
        } else {
            double t = 0.0;
            for (int p = 0; p < 8; ++p) t += r.part[k][p];
            r.tot[k] = t;
        }
    }
    __syncthreads();
    return true;
}

// A member's share of an iteration of the tracking kernel (members are
// work-groups 0 .. groups-1): store the tagged work-group partial in its
// XCD's slot (at work-group scope when `local`: on the leader's XCD); the
// leader of each leaf adds the leaf's partials as they carry the tag and
// stores the tagged leaf sum (device scope).  False (in every thread of
// a leader) on timeout or abort.
template <bool COMP>
__device__ inline bool contribute(const float acc[kNE], const float cmp[kNE], double* part, double* leafpart,
                                  int groups, const unsigned* sync, unsigned max_polls, ReduceLds& r,
                                  unsigned long long tag, bool local) {
    const int b = blockIdx.x;
    double* mine = part + (size_t)((b % kXcds) * kPerXcd + b / kXcds) * kPartStride;
    store_partial<COMP>(acc, cmp, mine, r, tag, local);
    if (!xcd_leader(b)) return true;
    const int leaf = xcd_leaf(b);
    const int leaf_size = min(kXcdLeaf, (groups - b + kXcds - 1) / kXcds);
    if (!total_leaves<COMP>(mine, leaf_size, tag, sync, max_polls, r)) return false;
    // r.tot holds the leaf sum in every thread; lanes of wave 0 store it
    if (threadIdx.x < kNE)
        __hip_atomic_store(reinterpret_cast<unsigned long long*>(&leafpart[(size_t)leaf * kPartStride + threadIdx.x]),
                           tag_word(r.tot[threadIdx.x], tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Wait (thread 0 only) until the sync word `word` reaches `target`;
// device-scope polling with a short sleep.  Returns false on timeout or when
// another work-group aborted.
__device__ inline bool wait_done(unsigned* sync, int word, unsigned target, unsigned max_polls) {
    unsigned spins = 0;
    while (__hip_atomic_load(&sync[word], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > max_polls ||
            __hip_atomic_load(&sync[kSyncAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Work-groups that take part at a level: about kPixPerGroup pixels each,
// at least kMinGroups (so coarse levels keep enough memory parallelism and
// a two-level tree) and at most the grid.  Measured on MI355X at 640x480
// (levels of 19200, 76800 and 307200 pixels): 128, 256 and 256 members per
// level; 64 at the coarsest level, or 128 at the middle one, are slower.
constexpr int kPixPerGroup = 256;
constexpr int kMinGroups = 128;
__device__ inline int level_groups(const TrackLevel& L, int G) {
    int g = (L.W * L.H + kPixPerGroup - 1) / kPixPerGroup;
    g = g < kMinGroups ? kMinGroups : g;
    return g > G ? G : g;
}

// Rank in the image of member b of n: the members split the level's pixels
// into n contiguous chunks, and band_rank (XCD-aware order of work-groups)
// orders them so that the members on one XCD take neighbouring chunks; each
// L2 then holds the voxels seen by one band of the image instead of the
// whole visible map.

// The whole coarse-to-fine Gauss-Newton of one frame (one launch, one work-group per CU).
//
// Only the members of a level (the first Gl work-groups) run its
// iterations; a work-group that joins at a later level takes the pose that
// work-group 0 publishes at the end of the previous level (it publishes only
// when the next level has more members).  Buffer reuse: partials and leaf
// sums alternate between two sets by iteration parity.  A member writes set
// (gi & 1) again at gi + 2 only after it has seen every leaf sum of gi + 1;
// each of those was published after its leaf's members had contributed to
// gi + 1, which they do only after reading the sums of gi, and by the first
// work-group of the leaf after it had read the leaf's partials of gi, so no
// set is read while it is overwritten.  The published pose of a level
// boundary is overwritten only at the next boundary, which needs the
// contributions of the work-groups that joined and read it.
template <int STORAGE, int MODEL>
__global__ __launch_bounds__(kTrackBlock) void k_track_frame(MapView M, TrackArgs a, const double* pose_in,
                                                              double* pose_out, double* partials, unsigned* sync,
                                                              float* stats, int32_t* status) {
    __shared__ double s_pose[12];
    __shared__ int s_ok, s_local;
    __shared__ ReduceLds red;
    __shared__ float s_depth[kTrackBatch * kTrackBlock];
    constexpr bool COMP = STORAGE == GSDF_BF16 || STORAGE == GSDF_FP16;
    const int G = gridDim.x;
    double* pose_pub = partials + 2 * kPartsPerSet;
    // a work-group that takes part in no level holds nothing anyone needs
    int span = 1;
    for (int l = 0; l < a.levels; ++l)
        if (a.iters[l] > 0) span = max(span, level_groups(a.lv[l], G));
    if ((int)blockIdx.x >= span) return;
    // the leaders publish their XCD; a member compares it with its own
    // before its first partial (at that point the leader's store has long
    // been visible, so the comparison costs one load)
    const bool leader = xcd_leader(blockIdx.x);
    if (leader && threadIdx.x == 0)
        __hip_atomic_store(&sync[kSyncXcc + xcd_leaf(blockIdx.x)], xcc_id() + 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    int local = a.device_scope ? 0 : (leader ? 1 : -1);   // -1: not known yet
    // pose_in may be pose_out: every work-group still running reads it here,
    // before its first contribution, and work-group 0 writes the result only
    // after the last iteration, which needs all of those contributions
    if (threadIdx.x < 12) s_pose[threadIdx.x] = pose_in[threadIdx.x];
    __syncthreads();
    if (!pose_finite(s_pose)) {
        // every work-group reads the same pose and leaves here: no iteration
        // runs, the estimate is the initial pose and the call reports it
        if (blockIdx.x == 0 && threadIdx.x < 12) pose_out[threadIdx.x] = s_pose[threadIdx.x];
        if (blockIdx.x == 0 && threadIdx.x == 0) raise_status(status, GSDF_EINVAL);
        return;
    }
    int gi = 0;           // global iteration index
    int have = 0;         // iterations the pose in s_pose reflects
    // per-iteration stamps (work-group 0, thread 0), when asked for
    const bool stamp = a.clocks && blockIdx.x == 0 && threadIdx.x == 0;
    const unsigned long long t0 = stamp ? wall_clock64() : 0ull;
    for (int l = a.levels - 1; l >= 0; --l) {
        if (a.iters[l] == 0) continue;
        const TrackLevel L = a.lv[l];
        const int Gl = level_groups(L, G);
        const int nleaf = xcd_leaves(Gl);
        if ((int)blockIdx.x >= Gl) {
            // not a member: skip the level
            gi += a.iters[l];
            continue;
        }
        if (have < gi) {
            // joining: take the pose published at the end of the previous level
            if (threadIdx.x == 0) s_ok = wait_done(sync, kSyncPub, (unsigned)gi, a.join_polls) ? 1 : 0;
            __syncthreads();
            if (!s_ok) {
                if (threadIdx.x == 0) {
                    __hip_atomic_store(&sync[kSyncAbort], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    raise_status(status, GSDF_EHIP);
                }
                return;
            }
            if (threadIdx.x < 12)
                s_pose[threadIdx.x] =
                    __hip_atomic_load(&pose_pub[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            have = gi;
        }
        // a member's pixels are one contiguous chunk of the level, the same
        // in every iteration: the depths of each thread's first batch are
        // loaded once and kept in LDS (each thread reads back only what it
        // wrote)
        const int npx = L.W * L.H;
        const int chunk = (npx + Gl - 1) / Gl;
        const int c0 = min(band_rank(blockIdx.x, Gl) * chunk, npx);
        const int c1 = min(c0 + chunk, npx);
        const int first = c0 + threadIdx.x;
#pragma unroll
        for (int j = 0; j < kTrackBatch; ++j) {
            const int i = first + j * kTrackBlock;
            s_depth[j * kTrackBlock + threadIdx.x] = i < c1 ? L.depth[i] : 0.0f;
        }
        for (int it = 0; it < a.iters[l]; ++it, ++gi) {
            double* part = partials + (size_t)(gi & 1) * kPartsPerSet;
            double* leafpart = part + (size_t)kMaxGroups * kPartStride;
            double P[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) P[k] = s_pose[k];
            float acc[kNE], cmp[kNE];
            if constexpr (MODEL == GSDF_MODEL_TRILINEAR)
                accumulate_trilinear<STORAGE>(M, L, a, P, first, kTrackBlock, c1, s_depth, acc, cmp);
            else
                accumulate<STORAGE>(M, L, a, P, first, kTrackBlock, c1, s_depth, acc, cmp);
            const unsigned long long tag = (unsigned long long)(gi + 1);
            if (stamp) a.clocks[4 * gi] = wall_clock64() - t0;
            if (local < 0) {
                // on the leader's XCD?  A bounded wait; if it ends without an
                // answer the partials simply go through device scope
                if (threadIdx.x == 0) {
                    const unsigned* w = &sync[kSyncXcc + xcd_leaf(blockIdx.x)];
                    unsigned v, spins = 0;
                    while ((v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0u &&
                           ++spins <= a.tag_polls)
                        __builtin_amdgcn_s_sleep(1);
                    s_local = v == xcc_id() + 1u ? 1 : 0;
                }
                __syncthreads();
                local = s_local;
            }
            // every member: the same sum of the leaf sums, the same solve
            const bool part_ok =
                contribute<COMP>(acc, cmp, part, leafpart, Gl, sync, a.tag_polls, red, tag, local != 0);
            if (stamp) a.clocks[4 * gi + 1] = wall_clock64() - t0;
            if (!part_ok || !total_leaves<COMP>(leafpart, nleaf, tag, sync, a.tag_polls, red)) {
                if (threadIdx.x == 0) {
                    __hip_atomic_store(&sync[kSyncAbort], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    raise_status(status, GSDF_EHIP);
                }
                return;
            }
            if (stamp) a.clocks[4 * gi + 2] = wall_clock64() - t0;
            if (threadIdx.x < 64) {
                const bool solved = solve_update_wave(red.tot, a.damping, s_pose);
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    const double* t = red.tot;
                    if (!solved) raise_status(status, GSDF_ENOTPD);
                    if (l == 0 && it == a.iters[0] - 1 && t[28] < (double)a.min_inlier_frac * t[29])
                        raise_status(status, GSDF_ELOST);
                    if (stats) {
                        stats[2 * gi] = (float)t[27];
                        stats[2 * gi + 1] = (float)t[28];
                    }
                    add_stat(M, kStatTrackValid, (unsigned long long)t[29]);
                    add_stat(M, kStatTrackUsed, (unsigned long long)t[28]);
                    if (stamp) a.clocks[4 * gi + 3] = wall_clock64() - t0;
                }
            }
            __syncthreads();
        }
        have = gi;
        // publish for the work-groups that join at the next level
        int next_groups = 0;
        for (int n = l - 1; n >= 0; --n)
            if (a.iters[n] > 0) {
                next_groups = level_groups(a.lv[n], G);
                break;
            }
        if (blockIdx.x == 0 && next_groups > Gl) {
            if (threadIdx.x < 12)
                __hip_atomic_store(&pose_pub[threadIdx.x], s_pose[threadIdx.x], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            if (threadIdx.x == 0) {
                complete_device_stores();
                __hip_atomic_store(&sync[kSyncPub], (unsigned)gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 12) pose_out[threadIdx.x] = s_pose[threadIdx.x];
}

// One linearisation (gsdf_normal_equations): a single launch whose last
// work-group writes the float64 totals.
template <int STORAGE>
__global__ __launch_bounds__(kTrackBlock) void k_normal_equations(MapView M, TrackArgs a,
                                                                   const double* pose, double* partials,
                                                                   unsigned* sync, double* out29) {
    __shared__ int s_last;
    __shared__ ReduceLds red;
    double P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = pose[k];
    float acc[kNE], cmp[kNE];
    accumulate<STORAGE>(M, a.lv[0], a, P, blockIdx.x * kTrackBlock + threadIdx.x, gridDim.x * kTrackBlock,
                        a.lv[0].W * a.lv[0].H, nullptr, acc, cmp);
    double ne[kNE];
    if (!reduce_tree<STORAGE != GSDF_FP32>(acc, cmp, partials, partials + (size_t)kMaxGroups * kPartStride, sync,
                                           0, gridDim.x, ne, red, &s_last))
        return;
    if (threadIdx.x == 0)
        for (int k = 0; k < 29; ++k) out29[k] = ne[k];
}

// One damped Gauss-Newton step at full resolution for each of K keyframes
// (the step k_track_frame takes with one level and one iteration), in two
// launches.  k_gn_partials: work-group (b, k) accumulates the normal
// equations of its strided share of keyframe k's pixels (about 8 a
// thread) at pose k and
// stores its partial in slot k * gridDim.x + b.  k_gn_solve: work-group k
// adds keyframe k's partials in a fixed order and takes the solve and the
// left update of k_track_frame.  The keyframes' pixel work shares one
// launch, so a refinement step pays two launches instead of two per
// keyframe.
template <int STORAGE>
__global__ __launch_bounds__(kTrackBlock) void k_gn_partials(MapView M, TrackArgs a, const double* poses,
                                                            double* partials) {
    __shared__ ReduceLds red;
    constexpr bool COMP = STORAGE == GSDF_BF16 || STORAGE == GSDF_FP16;
    const int k = blockIdx.y;
    double P[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) P[i] = poses[12 * k + i];
    TrackLevel L = a.lv[0];
    const int npx = L.W * L.H;
    L.depth += (size_t)k * npx;
    float acc[kNE], cmp[kNE];
    if (pose_finite(P)) {
        accumulate<STORAGE>(M, L, a, P, blockIdx.x * kTrackBlock + threadIdx.x, gridDim.x * kTrackBlock, npx,
                            nullptr, acc, cmp);
    } else {
        // the solve leaves this keyframe as it is and reports it
#pragma unroll
        for (int e = 0; e < kNE; ++e) acc[e] = cmp[e] = 0.0f;
    }
    store_partial<COMP>(acc, cmp, partials + ((size_t)k * gridDim.x + blockIdx.x) * kPartStride, red);
}

template <int STORAGE>
__global__ __launch_bounds__(kTrackBlock) void k_gn_solve(MapView M, double* poses, const double* partials,
                                                         int groups, double damping, float min_inlier_frac,
                                                         int32_t* status) {
    __shared__ ReduceLds red;
    __shared__ double s_pose[12];
    constexpr bool COMP = STORAGE == GSDF_BF16 || STORAGE == GSDF_FP16;
    const int k = blockIdx.x;
    if (threadIdx.x < 12) s_pose[threadIdx.x] = poses[12 * k + threadIdx.x];
    __syncthreads();
    if (!pose_finite(s_pose)) {   // the same pose for every thread: a uniform exit
        if (threadIdx.x == 0) raise_status(status, GSDF_EINVAL);
        return;
    }
    double ne[kNE];
    total_partials<COMP>(partials + (size_t)k * groups * kPartStride, groups, ne, red);
    if (threadIdx.x < 64) {
        const bool solved = solve_update_wave(red.tot, damping, s_pose);
        if (threadIdx.x == 0) {
            const double* t = red.tot;
            if (!solved) raise_status(status, GSDF_ENOTPD);
            if (t[28] < (double)min_inlier_frac * t[29]) raise_status(status, GSDF_ELOST);
            add_stat(M, kStatTrackValid, (unsigned long long)t[29]);
            add_stat(M, kStatTrackUsed, (unsigned long long)t[28]);
        }
    }
    __syncthreads();
    if (threadIdx.x < 12) poses[12 * k + threadIdx.x] = s_pose[threadIdx.x];
}

// All pyramid levels in one launch, each by the 2x2 rule in binary32: the
// mean of four valid depths whose spread is within the truncation, else 0.
// A work-group covers a 16x16 tile of level 1 (from level 0 in global
// memory); its 8x8 level-2 and 4x4 level-3 pixels come from LDS.  The
// work-groups also clear the sync words and the tagged partials and leaf
// sums of the tracking kernel between them.
struct PyramidArgs {
    const float* src;
    float* dst[4];
    int W[4], H[4];
    int levels;
    float zmin, zmax, Tf;
    unsigned* sync;
    unsigned long long* sets[2];   // tagged partials and leaf sums of the two sets (null: none)
    int part_words;                // words of the work-group partials of a set to clear
};

__device__ inline float pyr_combine(float a, float b, float c, float e, const PyramidArgs& p) {
    bool ok = depth_ok(a, p.zmin, p.zmax) && depth_ok(b, p.zmin, p.zmax) && depth_ok(c, p.zmin, p.zmax) &&
              depth_ok(e, p.zmin, p.zmax);
    const float mx = fmaxf(fmaxf(a, b), fmaxf(c, e));
    const float mn = fminf(fminf(a, b), fminf(c, e));
    ok = ok && (sub_rn(mx, mn) <= p.Tf);
    return ok ? mul_rn(add_rn(add_rn(a, b), add_rn(c, e)), 0.25f) : 0.0f;
}

__global__ __launch_bounds__(256) void k_pyramid(PyramidArgs p) {
    __shared__ float t1[16][17];
    __shared__ float t2[8][9];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    {
        // every work-group clears its share of the tracking kernel's sync
        // words and tagged words
        const int nthreads = gridDim.x * gridDim.y * blockDim.x;
        const int tid = (blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
        for (int k = tid; k < kSyncWords; k += nthreads) p.sync[k] = 0u;
        if (p.sets[0]) {
            // the partials of the work-groups that run, then every leaf sum
            constexpr int kLeafWords = kMaxLeaves * kPartStride;
            for (int k = tid; k < p.part_words + kLeafWords; k += nthreads) {
                const size_t w = k < p.part_words ? (size_t)k
                                                  : (size_t)kMaxGroups * kPartStride + (size_t)(k - p.part_words);
                p.sets[0][w] = 0ull;
                p.sets[1][w] = 0ull;
            }
        }
    }
    if (p.levels < 2) return;
    const int u = blockIdx.x * 16 + tx, v = blockIdx.y * 16 + ty;
    float d1 = 0.0f;
    if (u < p.W[1] && v < p.H[1]) {
        const float* r0 = p.src + (size_t)(2 * v) * p.W[0] + 2 * u;
        const float* r1 = r0 + p.W[0];
        d1 = pyr_combine(r0[0], r0[1], r1[0], r1[1], p);
        p.dst[1][(size_t)v * p.W[1] + u] = d1;
    }
    t1[ty][tx] = d1;
    if (p.levels < 3) return;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int a = threadIdx.x & 7, b = threadIdx.x >> 3;
        const int u2 = blockIdx.x * 8 + a, v2 = blockIdx.y * 8 + b;
        float d2 = 0.0f;
        if (u2 < p.W[2] && v2 < p.H[2]) {
            d2 = pyr_combine(t1[2 * b][2 * a], t1[2 * b][2 * a + 1], t1[2 * b + 1][2 * a],
                             t1[2 * b + 1][2 * a + 1], p);
            p.dst[2][(size_t)v2 * p.W[2] + u2] = d2;
        }
        t2[b][a] = d2;
    }
    if (p.levels < 4) return;
    __syncthreads();
    if (threadIdx.x < 16) {
        const int a = threadIdx.x & 3, b = threadIdx.x >> 2;
        const int u3 = blockIdx.x * 4 + a, v3 = blockIdx.y * 4 + b;
        if (u3 < p.W[3] && v3 < p.H[3])
            p.dst[3][(size_t)v3 * p.W[3] + u3] =
                pyr_combine(t2[2 * b][2 * a], t2[2 * b][2 * a + 1], t2[2 * b + 1][2 * a], t2[2 * b + 1][2 * a + 1], p);
    }
}

struct ScratchLayout {
    size_t sync, partials, level[4], total;
};

inline ScratchLayout scratch_layout(const gsdf_camera& c, int levels) {
    ScratchLayout s;
    size_t o = 0;
    s.sync = o;     o = align256(o + kSyncWords * 4);
    s.partials = o; o = align256(o + (2 * kPartsPerSet + 16) * 8);  // two sets, then the published pose
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

// Keyframes of one batched Gauss-Newton step (the grid's y extent).
constexpr int kMaxGnKeyframes = 65535;

// Work-groups per keyframe of the batched Gauss-Newton step: about 8
// pixels a thread, so the work-group's fixed costs (its partial's LDS sum
// and store) are shared by more pixels.  Measured at 30 keyframes of
// 640x480: 190 us at 2 pixels a thread, 160 at 4, 138 at 8, 132 at 16
// (which leaves most CUs idle below about 8 keyframes).
inline int gn_groups(int npx) {
    const int g = ceil_div(npx, kTrackBlock * 8);
    return g < 1 ? 1 : (g > kMaxGroups ? kMaxGroups : g);
}

inline int normal_eq_groups(int npx) {
    int g = ceil_div(npx, kTrackBlock * 2);   // about two pixels per thread
    return g < 1 ? 1 : (g > kMaxGroups ? kMaxGroups : g);
}

// Work-group count of the tracking kernel: one per CU of the current
// device (queried on every call; the runtime answers from its own device
// table).  The work-groups wait for each other, so all of them must be
// resident at once.  A work-group needs 512 threads (two waves per SIMD) and
// less LDS than a CU holds (checked below at compile time), so an idle CU
// always takes one.  The kernel is launched like any other on the stream (a
// cooperative launch costs about 15 us more per frame in dispatch, measured
// on MI355X): on a device that other work keeps partly busy the last
// work-groups start late, and every wait is bounded, so the worst case is a
// frame that fails with GSDF_EHIP.
constexpr size_t kTrackLds = sizeof(ReduceLds) + sizeof(float) * kTrackBatch * kTrackBlock + 16 * sizeof(double);
static_assert(kTrackLds <= 160 * 1024, "the tracking work-group must fit one CU's LDS (160 KB on gfx950)");
inline int track_groups() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus < kMaxGroups ? cus : kMaxGroups;
}

template <int STORAGE, int MODEL>
int launch_track_frame(gsdf_timer* timer, hipStream_t s, const MapView& M, const TrackArgs& a,
                       const double* pose_in, double* pose_out, double* partials, unsigned* sync, float* stats,
                       int32_t* status) {
    const int g = track_groups();
    if (g <= 0) return GSDF_EHIP;
    TimedLaunch tl(timer, GSDF_K_TRACK, s);
    k_track_frame<STORAGE, MODEL><<<g, kTrackBlock, 0, s>>>(M, a, pose_in, pose_out, partials, sync, stats,
                                                            status);
    return GSDF_OK;
}

template <int STORAGE>
int launch_track_model(int model, gsdf_timer* timer, hipStream_t s, const MapView& M, const TrackArgs& a,
                       const double* pose_in, double* pose_out, double* partials, unsigned* sync, float* stats,
                       int32_t* status) {
    if (model == GSDF_MODEL_TRILINEAR)
        return launch_track_frame<STORAGE, GSDF_MODEL_TRILINEAR>(timer, s, M, a, pose_in, pose_out, partials,
                                                                sync, stats, status);
    if constexpr (STORAGE == GSDF_NOGRAD_FP32) {
        return GSDF_EINVAL;   // the Taylor model needs the stored gradient
    } else {
        return launch_track_frame<STORAGE, GSDF_MODEL_TAYLOR>(timer, s, M, a, pose_in, pose_out, partials, sync,
                                                             stats, status);
    }
}

inline void fill_levels(const gsdf_camera& cam, const float* depth, const ScratchLayout& sl, char* base,
                        int levels, TrackArgs* a) {
    double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
    a->lv[0].depth = depth;
    a->lv[0].W = cam.width;
    a->lv[0].H = cam.height;
    a->lv[0].ifx = 1.0 / fx;
    a->lv[0].ify = 1.0 / fy;
    a->lv[0].cx = cx;
    a->lv[0].cy = cy;
    for (int l = 1; l < 4; ++l) {
        fx /= 2;
        fy /= 2;
        cx = (cx + 0.5) / 2 - 0.5;
        cy = (cy + 0.5) / 2 - 0.5;
        a->lv[l].depth = l < levels ? (const float*)(base + sl.level[l]) : nullptr;
        a->lv[l].W = a->lv[l - 1].W / 2;
        a->lv[l].H = a->lv[l - 1].H / 2;
        a->lv[l].ifx = 1.0 / fx;
        a->lv[l].ify = 1.0 / fy;
        a->lv[l].cx = cx;
        a->lv[l].cy = cy;
    }
}

}  // namespace gsdf

using namespace gsdf;

extern "C" int gsdf_wall_clock_khz(int32_t* khz_out) {
    if (!khz_out) return GSDF_EINVAL;
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return GSDF_EHIP;
    *khz_out = khz;
    return GSDF_OK;
}

extern "C" size_t gsdf_track_scratch_bytes(const gsdf_camera* cam, int32_t levels) {
    if (!valid_cam(cam) || levels < 1 || levels > 4) return 0;
    return scratch_layout(*cam, levels).total;
}

namespace gsdf {

// gsdf_track_frame on a given scratch buffer (the caller's, or the
// library's fixed array for gsdf_track_frame_noalloc).
int track_frame_on(const gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                   const gsdf_track_params* params, const double* T_init_dev, double* T_wc_out_dev, float* stats_dev,
                   void* scratch_dev, size_t scratch_bytes, int32_t* status_dev, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !params || !T_init_dev || !T_wc_out_dev ||
        !scratch_dev)
        return GSDF_EINVAL;
    const int levels = params->levels;
    if (levels < 1 || levels > 4) return GSDF_EINVAL;
    for (int l = 0; l < levels; ++l)
        if (params->iters[l] < 0 || params->iters[l] > 1000) return GSDF_EINVAL;
    if (params->model != GSDF_MODEL_TAYLOR && params->model != GSDF_MODEL_TRILINEAR) return GSDF_EINVAL;
    if (params->max_polls < 0) return GSDF_EINVAL;
    if (params->model == GSDF_MODEL_TAYLOR && !has_gradients(map)) return GSDF_EINVAL;
    if ((cam->width >> (levels - 1)) < 1 || (cam->height >> (levels - 1)) < 1) return GSDF_EINVAL;
    const ScratchLayout sl = scratch_layout(*cam, levels);
    if (scratch_bytes < sl.total) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)scratch_dev;
    unsigned* sync = (unsigned*)(base + sl.sync);
    double* partials = (double*)(base + sl.partials);

    TrackArgs a;
    fill_levels(*cam, depth_dev, sl, base, levels, &a);
    a.levels = levels;
    for (int l = 0; l < 4; ++l) a.iters[l] = l < levels ? params->iters[l] : 0;
    a.zmin = cam->zmin;
    a.zmax = cam->zmax;
    a.delta = params->huber_delta;
    a.inv_vs = 1.0 / map->desc.voxel_size;
    a.vs = map->desc.voxel_size;
    a.damping = params->damping;
    a.min_inlier_frac = params->min_inlier_frac;
    a.tag_polls = params->max_polls > 0 ? (unsigned)params->max_polls : kTagPolls;
    a.join_polls = params->max_polls > 0 ? (unsigned)params->max_polls : kJoinPolls;
    a.clocks = reinterpret_cast<unsigned long long*>(params->iter_clocks);
    a.device_scope = params->exchange_device_scope ? 1 : 0;

    {
        PyramidArgs p;
        p.src = depth_dev;
        for (int l = 0; l < 4; ++l) {
            p.dst[l] = (float*)a.lv[l].depth;
            p.W[l] = a.lv[l].W;
            p.H[l] = a.lv[l].H;
        }
        p.levels = levels;
        p.zmin = cam->zmin;
        p.zmax = cam->zmax;
        p.Tf = (float)map->desc.truncation;
        p.sync = sync;
        for (int q = 0; q < 2; ++q)
            p.sets[q] = reinterpret_cast<unsigned long long*>(partials + (size_t)q * kPartsPerSet);
        p.part_words = kMaxGroups * kPartStride;
        TimedLaunch tp(map->timer, GSDF_K_PYRAMID, s);
        // a single level has no pyramid work: enough work-groups for the clearing
        dim3 grd(levels > 1 ? ceil_div(a.lv[1].W, 16) : 32, levels > 1 ? ceil_div(a.lv[1].H, 16) : 1);
        k_pyramid<<<grd, 256, 0, s>>>(p);
    }
    const MapView M = make_view(*map);
    int rc;
    switch (map->desc.storage) {
        case GSDF_FP32: rc = launch_track_model<GSDF_FP32>(params->model, map->timer, s, M, a, T_init_dev, T_wc_out_dev, partials, sync, stats_dev, status_dev); break;
        case GSDF_BF16: rc = launch_track_model<GSDF_BF16>(params->model, map->timer, s, M, a, T_init_dev, T_wc_out_dev, partials, sync, stats_dev, status_dev); break;
        case GSDF_FP16: rc = launch_track_model<GSDF_FP16>(params->model, map->timer, s, M, a, T_init_dev, T_wc_out_dev, partials, sync, stats_dev, status_dev); break;
        default: rc = launch_track_model<GSDF_NOGRAD_FP32>(params->model, map->timer, s, M, a, T_init_dev, T_wc_out_dev, partials, sync, stats_dev, status_dev); break;
    }
    if (rc != GSDF_OK) return rc;
    return launch_status();
}

// Scratch of gsdf_track_frame_noalloc: one file-scope device array, which
// each GPU the library runs on holds until the process ends.  Its host-side
// name is only a handle for the runtime: kernels receive the device address
// that hipGetSymbolAddress returns for the current device, looked up once
// per device and kept.
constexpr size_t kNoAllocScratch = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, or nullptr.
void* noalloc_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace gsdf

extern "C" int gsdf_track_frame(const gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                                const gsdf_track_params* params, const double* T_init_dev, double* T_wc_out_dev,
                                float* stats_dev, void* scratch_dev, size_t scratch_bytes,
                                int32_t* status_dev, void* stream) {
    return track_frame_on(map, depth_dev, cam, params, T_init_dev, T_wc_out_dev, stats_dev, scratch_dev,
                          scratch_bytes, status_dev, stream);
}

extern "C" size_t gsdf_track_noalloc_max_bytes(void) { return kNoAllocScratch; }

extern "C" int gsdf_track_frame_noalloc(const gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                                        const gsdf_track_params* params, const double* T_init_dev,
                                        double* T_wc_out_dev, float* stats_dev, int32_t* status_dev,
                                        void* stream) {
    if (!valid_cam(cam) || !params || params->levels < 1 || params->levels > 4) return GSDF_EINVAL;
    if (scratch_layout(*cam, params->levels).total > kNoAllocScratch) return GSDF_EINVAL;
    void* base = noalloc_scratch();
    if (!base) return GSDF_EHIP;
    return track_frame_on(map, depth_dev, cam, params, T_init_dev, T_wc_out_dev, stats_dev, base, kNoAllocScratch,
                          status_dev, stream);
}

extern "C" int gsdf_normal_equations(const gsdf_map* map, const float* depth_dev,
                                     const gsdf_camera* cam, const double* T_wc_dev,
                                     float huber_delta, double* out29_dev, void* scratch_dev,
                                     size_t scratch_bytes, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !T_wc_dev || !out29_dev || !scratch_dev)
        return GSDF_EINVAL;
    if (!has_gradients(map)) return GSDF_EINVAL;
    const ScratchLayout sl = scratch_layout(*cam, 1);
    if (scratch_bytes < sl.total) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)scratch_dev;
    unsigned* sync = (unsigned*)(base + sl.sync);
    double* partials = (double*)(base + sl.partials);
    TrackArgs a;
    fill_levels(*cam, depth_dev, sl, base, 1, &a);
    a.levels = 1;
    a.zmin = cam->zmin;
    a.zmax = cam->zmax;
    a.delta = huber_delta;
    a.inv_vs = 1.0 / map->desc.voxel_size;
    a.vs = map->desc.voxel_size;
    a.damping = 0.0;
    a.min_inlier_frac = 0.0f;
    a.tag_polls = kTagPolls;
    a.join_polls = kJoinPolls;
    a.clocks = nullptr;
    a.device_scope = 1;
    PyramidArgs p = {};
    p.levels = 1;
    p.sync = sync;
    k_pyramid<<<1, 256, 0, s>>>(p);
    const int g = normal_eq_groups(cam->width * cam->height);
    const MapView M = make_view(*map);
    switch (map->desc.storage) {
        case GSDF_FP32: k_normal_equations<GSDF_FP32><<<g, kTrackBlock, 0, s>>>(M, a, T_wc_dev, partials, sync, out29_dev); break;
        case GSDF_BF16: k_normal_equations<GSDF_BF16><<<g, kTrackBlock, 0, s>>>(M, a, T_wc_dev, partials, sync, out29_dev); break;
        default: k_normal_equations<GSDF_FP16><<<g, kTrackBlock, 0, s>>>(M, a, T_wc_dev, partials, sync, out29_dev); break;
    }
    return launch_status();
}

extern "C" size_t gsdf_gn_scratch_bytes(const gsdf_camera* cam, int32_t n_keyframes) {
    if (!valid_cam(cam) || n_keyframes <= 0 || n_keyframes > kMaxGnKeyframes) return 0;
    return align256((size_t)n_keyframes * gn_groups(cam->width * cam->height) * kPartStride *
                    sizeof(double));
}

extern "C" int gsdf_gn_step_keyframes(const gsdf_map* map, const float* depth_dev, int32_t n_keyframes,
                                      const gsdf_camera* cam, double* T_dev, float huber_delta, double damping,
                                      float min_inlier_frac, void* scratch_dev, size_t scratch_bytes,
                                      int32_t* status_dev, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !T_dev || !scratch_dev || !status_dev)
        return GSDF_EINVAL;
    if (n_keyframes <= 0 || n_keyframes > kMaxGnKeyframes) return GSDF_EINVAL;
    if (!(huber_delta > 0.0f) || !(damping >= 0.0)) return GSDF_EINVAL;
    if (!has_gradients(map)) return GSDF_EINVAL;
    if (scratch_bytes < gsdf_gn_scratch_bytes(cam, n_keyframes)) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const ScratchLayout sl = scratch_layout(*cam, 1);
    TrackArgs a;
    fill_levels(*cam, depth_dev, sl, nullptr, 1, &a);
    a.levels = 1;
    for (int l = 0; l < 4; ++l) a.iters[l] = l == 0 ? 1 : 0;
    a.zmin = cam->zmin;
    a.zmax = cam->zmax;
    a.delta = huber_delta;
    a.inv_vs = 1.0 / map->desc.voxel_size;
    a.vs = map->desc.voxel_size;
    a.damping = damping;
    a.min_inlier_frac = min_inlier_frac;
    a.tag_polls = kTagPolls;
    a.join_polls = kJoinPolls;
    a.clocks = nullptr;
    a.device_scope = 1;
    const int g = gn_groups(cam->width * cam->height);
    const dim3 grid(g, n_keyframes);
    double* partials = (double*)scratch_dev;
    const MapView M = make_view(*map);
    switch (map->desc.storage) {
        case GSDF_FP32:
            k_gn_partials<GSDF_FP32><<<grid, kTrackBlock, 0, s>>>(M, a, T_dev, partials);
            k_gn_solve<GSDF_FP32><<<n_keyframes, kTrackBlock, 0, s>>>(M, T_dev, partials, g, damping, min_inlier_frac,
                                                                     status_dev);
            break;
        case GSDF_BF16:
            k_gn_partials<GSDF_BF16><<<grid, kTrackBlock, 0, s>>>(M, a, T_dev, partials);
            k_gn_solve<GSDF_BF16><<<n_keyframes, kTrackBlock, 0, s>>>(M, T_dev, partials, g, damping, min_inlier_frac,
                                                                     status_dev);
            break;
        default:
            k_gn_partials<GSDF_FP16><<<grid, kTrackBlock, 0, s>>>(M, a, T_dev, partials);
            k_gn_solve<GSDF_FP16><<<n_keyframes, kTrackBlock, 0, s>>>(M, T_dev, partials, g, damping, min_inlier_frac,
                                                                     status_dev);
            break;
    }
    return launch_status();
}
