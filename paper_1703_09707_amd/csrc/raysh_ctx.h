// The context behind the opaque raysh_ctx handle, and the host helpers the
// C-ABI sources share (validation, error strings, parameter packing).
#pragma once

#include "raysh_internal.h"

struct raysh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n_stars = 0;
    raysh::Star *d_stars = nullptr;        // n_stars records (at least one allocated)
    int64_t star_capacity = 0;             // records d_stars holds
    raysh::Star *h_stage[2] = {nullptr, nullptr};   // pinned staging of star uploads, kept for raysh_set_lens
    size_t stage_records = 0;              // records each staging buffer holds
    double kappa_c = 0, gamma1 = 0, gamma2 = 0;
    double k11 = 0, k12 = 0, k22 = 0;      // K of Eq. (3)
    unsigned long long *d_counter = nullptr;
    unsigned long long *h_counter = nullptr;   // pinned
    // default launch shapes: the fastest on MI355X for the 16384-star workload
    raysh::TileShape shape[2] = {{8, 4, 16, 1}, {4, 4, 0, 128}};
    int star_parts = 1;                    // FP64 split of each ray's star sum (0 = automatic)
    double theta_open = 0.25;              // far-star criterion of RAYSH_FP64_EXPANSION
    int expansion_block = 0;               // tiles per side of its workgroups (0 = automatic)
    int expansion_cells = RAYSH_CELLS_AUTO;   // star cells of its block pass
    bool cells_built = false;
    raysh::StarCellStore cells;            // built on the first call that uses them
    double2 *d_partial = nullptr;          // split-K workspace
    size_t partial_bytes = 0;
    void *d_far = nullptr;                 // expansion mode: the blocks' coefficients and near lists
    size_t far_bytes = 0;
    int n_cu = 0;
};

// Error reporting: store a message for raysh_last_error and return code.
int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);
int set_ok();

// Validation (no device calls except validate_device_ptr).
int validate_rays(const raysh_rays *r);
int validate_pixels(const raysh_pixels *p);
int validate_precision(int precision);
int validate_tiled_precision(int precision);   // RAYSH_FP64 or RAYSH_FP32_BULK only
int validate_device_ptr(const void *ptr, size_t bytes, int device, const char *name);

// Lens, rays and window of one call packed for the kernels (outputs unset).
void fill_shoot_params(raysh::ShootParams &p, const raysh_ctx *c, const raysh_rays *r,
                       const raysh_pixels *w);

// Drop captured batch launches that reference ctx (called by raysh_free).
void raysh_forget_batches(const raysh_ctx *ctx);

// Makes `dev` current for the scope and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
};
