// raysh_map_batch: many independent lenses (parameter sets) in one
// persistent launch, captured once into a HIP graph and replayed.
//
// Sec. 2.2 of arXiv:1703.09707 notes that grids of independent simulations
// over (<M>, gamma, kappa_*, kappa_c) are common; here they share one
// launch.  Work items are (set, run of consecutive ray tiles); sets are
// ordered by decreasing cost per tile (stars x rays per tile), so the queue
// hands out the longest items first and the short ones fill the tail.  Sets
// with few stars get several tiles per item so that every item carries
// about 2^25 ray-star interactions.
#include <algorithm>
#include <limits>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "raysh_internal.h"
#include "raysh_ctx.h"

using raysh::BatchArgs;
using raysh::BatchSet;
using raysh::ShootParams;
using raysh::TileShape;

namespace {

struct BatchPlan {
    int device = 0;
    int precision = 0;
    TileShape shape{};
    std::vector<const raysh_ctx *> ctxs;
    std::vector<raysh_rays> rays;
    std::vector<raysh_pixels> pix;
    std::vector<int32_t *> counts;
    BatchSet *d_sets = nullptr;
    unsigned long long *d_queue = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t total_items = 0;
    int blocks = 0;

    bool same(const raysh_ctx *const *s, int n, const raysh_rays *r, const raysh_pixels *p, int prec,
              int32_t *const *c, const TileShape &t) const {
        if ((int)ctxs.size() != n || prec != precision) return false;
        if (std::memcmp(&t, &shape, sizeof t) != 0) return false;
        for (int i = 0; i < n; ++i) {
            if (ctxs[i] != s[i] || counts[i] != c[i]) return false;
            if (std::memcmp(&rays[i], &r[i], sizeof(raysh_rays)) != 0) return false;
            if (std::memcmp(&pix[i], &p[i], sizeof(raysh_pixels)) != 0) return false;
        }
        return true;
    }

    bool uses(const raysh_ctx *c) const { return std::find(ctxs.begin(), ctxs.end(), c) != ctxs.end(); }

    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_sets) (void)hipFree(d_sets);
        if (d_queue) (void)hipFree(d_queue);
        exec = nullptr;
        graph = nullptr;
        d_sets = nullptr;
        d_queue = nullptr;
    }
};

constexpr int64_t kItemWork = int64_t(1) << 25;   // ray-star interactions per queue item

std::mutex g_mu;
std::vector<BatchPlan *> g_plans;   // most recently used last
constexpr size_t kMaxPlans = 8;

void drop_plan(BatchPlan *p) {
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();   // a replay may still be running
    p->release();
    delete p;
}

// Build the descriptor table, upload it and capture [queue reset, persistent
// kernel] into a graph.  Returns a RAYSH_* code.
int build_plan(BatchPlan *plan, raysh_ctx *const *sets, int n_sets, const raysh_rays *rays,
               const raysh_pixels *pix, int precision, int32_t *const *counts) {
    const TileShape t = plan->shape;
    const int tw = raysh::tile_width(t), th = raysh::tile_height(t);
    std::vector<int> order(n_sets);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return sets[a]->n_stars > sets[b]->n_stars;
    });
    std::vector<BatchSet> host;
    host.reserve(n_sets);
    int64_t items = 0;
    for (int s : order) {
        const raysh_rays &r = rays[s];
        if (r.nx == 0 || r.ny == 0) continue;
        BatchSet b{};
        fill_shoot_params(b.p, sets[s], &r, &pix[s]);
        b.p.counts = counts[s];
        const int64_t tx = (r.nx + tw - 1) / tw, ty = (r.ny + th - 1) / th;
        b.p.tiles_x = (int32_t)tx;
        b.n_tiles = tx * ty;
        // an item covers enough tiles for ~kItemWork ray-star interactions,
        // so the queue's atomic and barrier stay small beside the work
        const int64_t per_tile = (int64_t)tw * th * std::max<int64_t>(sets[s]->n_stars, 1);
        b.tiles_per_item = (int32_t)std::min<int64_t>(std::max<int64_t>(kItemWork / per_tile, 1), 64);
        b.first_item = items;
        b.n_items = (b.n_tiles + b.tiles_per_item - 1) / b.tiles_per_item;
        items += b.n_items;
        host.push_back(b);
    }
    plan->total_items = items;
    if (items == 0) return RAYSH_OK;
    if (items > std::numeric_limits<int32_t>::max())
        return set_error(RAYSH_EOVERFLOW, "raysh_map_batch: more than 2^31-1 work items");

    hipError_t e = hipMalloc(&plan->d_sets, host.size() * sizeof(BatchSet));
    if (e == hipSuccess) e = hipMalloc(&plan->d_queue, sizeof(unsigned long long));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_ENOMEM, "raysh_map_batch: device allocation failed");
    }
    e = hipMemcpy(plan->d_sets, host.data(), host.size() * sizeof(BatchSet), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "raysh_map_batch upload");

    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, plan->device);
    if (e != hipSuccess) return hip_error(e, "raysh_map_batch");
    const int per_cu = precision == RAYSH_FP64 ? raysh::batch_fp64_blocks_per_cu(t)
                                               : raysh::batch_fp32_blocks_per_cu(t);
    plan->blocks = (int)std::min<int64_t>((int64_t)ncu * per_cu, items);

    BatchArgs args{plan->d_sets, (int32_t)host.size(), items, plan->d_queue};
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_error(e, "raysh_map_batch stream");
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = raysh::launch_zero_u64(plan->d_queue, 1, cap);
        if (le == hipSuccess)
            le = precision == RAYSH_FP64 ? raysh::launch_batch_fp64(args, t, plan->blocks, cap)
                                         : raysh::launch_batch_fp32(args, t, plan->blocks, cap);
        e = hipStreamEndCapture(cap, &plan->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_error(e, "raysh_map_batch capture");
    return RAYSH_OK;
}

}  // namespace

void raysh_forget_batches(const raysh_ctx *ctx) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if ((*it)->uses(ctx)) {
            drop_plan(*it);
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
}

extern "C" int raysh_map_batch(raysh_ctx *const *sets, int n_sets, const raysh_rays *rays,
                               const raysh_pixels *pix, int precision, int32_t *const *counts) {
    if (!sets || !rays || !pix || !counts) return set_error(RAYSH_EINVAL, "raysh_map_batch: NULL array");
    if (n_sets < 1) return set_error(RAYSH_EINVAL, "raysh_map_batch: n_sets < 1");
    if (int r = validate_tiled_precision(precision)) return r;
    for (int s = 0; s < n_sets; ++s) {
        if (!sets[s]) return set_error(RAYSH_EINVAL, "raysh_map_batch: set %d has no context", s);
        if (sets[s]->device != sets[0]->device)
            return set_error(RAYSH_EINVAL, "raysh_map_batch: contexts on different devices");
        if (int r = validate_rays(&rays[s])) return r;
        if (int r = validate_pixels(&pix[s])) return r;
        if (!counts[s]) return set_error(RAYSH_EINVAL, "raysh_map_batch: counts[%d] is NULL", s);
    }
    raysh_ctx *lead = sets[0];
    DeviceGuard g(lead->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", lead->device);
    for (int s = 0; s < n_sets; ++s) {
        const size_t bytes = (size_t)pix[s].nx * (size_t)pix[s].ny * 4;
        if (int r = validate_device_ptr(counts[s], bytes, lead->device, "counts")) return r;
    }
    const TileShape t = lead->shape[precision];

    std::lock_guard<std::mutex> lk(g_mu);
    BatchPlan *plan = nullptr;
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
        if ((*it)->same(sets, n_sets, rays, pix, precision, counts, t)) {
            plan = *it;
            g_plans.erase(it);
            break;
        }
    }
    if (!plan) {
        plan = new BatchPlan();
        plan->device = lead->device;
        plan->precision = precision;
        plan->shape = t;
        plan->ctxs.assign(sets, sets + n_sets);
        plan->rays.assign(rays, rays + n_sets);
        plan->pix.assign(pix, pix + n_sets);
        plan->counts.assign(counts, counts + n_sets);
        int r = build_plan(plan, sets, n_sets, rays, pix, precision, counts);
        if (r != RAYSH_OK) {
            drop_plan(plan);
            return r;
        }
        if (g_plans.size() >= kMaxPlans) {
            drop_plan(g_plans.front());
            g_plans.erase(g_plans.begin());
        }
    }
    g_plans.push_back(plan);
    if (plan->total_items == 0) return set_ok();
    hipError_t e = hipGraphLaunch(plan->exec, lead->stream);
    if (e != hipSuccess) return hip_error(e, "raysh_map_batch launch");
    return set_ok();
}
