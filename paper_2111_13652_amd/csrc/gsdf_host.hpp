// Host-side helpers of libgsdf: argument checks, launch bracketing with the
// optional event timer, and camera/pose constants.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "gsdf_common.hpp"

namespace gsdf {

// ---- optional per-kernel event timing: the caller's gsdf_timer attached to
// the map (gsdf_map.timer; NULL = none) ----
bool timing_on(gsdf_timer* t, int kernel_id);
void timing_begin(gsdf_timer* t, int kernel_id, hipStream_t s);
void timing_end(gsdf_timer* t, int kernel_id, hipStream_t s);

struct TimedLaunch {
    gsdf_timer* t;
    int id;
    hipStream_t s;
    bool on;
    TimedLaunch(gsdf_timer* timer, int kernel_id, hipStream_t stream)
        : t(timer), id(kernel_id), s(stream), on(timer && timing_on(timer, kernel_id)) {
        if (on) timing_begin(t, id, s);
    }
    ~TimedLaunch() {
        if (on) timing_end(t, id, s);
    }
};

inline bool valid_desc(const gsdf_map_desc& d) {
    if (!(d.voxel_size > 0.0) || !(d.truncation >= d.voxel_size)) return false;
    if (d.max_blocks <= 0 || d.max_blocks > (1 << 24)) return false;
    if (d.hash_slots <= 0 || (d.hash_slots & (d.hash_slots - 1)) != 0) return false;
    if (d.hash_slots < d.max_blocks) return false;
    if (d.storage < GSDF_FP32 || d.storage > GSDF_NOGRAD_FP32) return false;
    return true;
}

inline bool valid_map(const gsdf_map* m) {
    return m && m->hash && m->vox && m->weight && m->aux && valid_desc(m->desc);
}

// Maps without stored gradients serve fusion and the tri-linear model only.
inline bool has_gradients(const gsdf_map* m) { return m->desc.storage != GSDF_NOGRAD_FP32; }

inline bool valid_cam(const gsdf_camera* c) {
    return c && c->width > 0 && c->height > 0 && c->width <= 16384 && c->height <= 16384 &&
           c->fx > 0 && c->fy > 0 && std::isfinite(c->cx) && std::isfinite(c->cy);
}

inline int launch_status() {
    return hipGetLastError() == hipSuccess ? GSDF_OK : GSDF_EHIP;
}

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace gsdf
