// Batched sweeps: many plans (e.g. the time frames of a sequence, each with
// its own grid and cameras) projected and backprojected by one persistent
// launch per direction, optionally captured once in a hipGraph and replayed.
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "ltm_internal.h"

namespace ltm {
namespace {

uint64_t align256(uint64_t v) { return (v + 255u) & ~uint64_t(255u); }

struct Dir {
    std::vector<uint32_t> items;   // (batch camera << kTileBits) | tile, by decreasing cost
    size_t lds = 0;                // dynamic LDS of the persistent kernel
    int blocks = 0;                // persistent workgroups
    uint64_t items_off = 0;
};

}  // namespace
}  // namespace ltm

struct ltm_batch {
    std::vector<ltm_plan*> plans;
    std::vector<std::pair<int, int>> pcs;     // (plan, camera) of each batch camera
    std::vector<ltm::BatchCam> host_cams[2];  // per direction (tilings differ)
    ltm::Dir dir[2];
    uint64_t cams_off[2] = {0, 0}, counter_off = 0, ws_bytes = 0;
    char* ws = nullptr;
    bool bound = false;
    // member plans' generations and view subsets when the work lists were
    // built (create) and when the tables were recorded (bind)
    std::vector<uint64_t> gen_create, gen_bind;
    std::vector<std::pair<uint32_t, uint32_t>> sub_bind;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace ltm {
namespace {

void release_graph(ltm_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// LTM_OK while every member plan still has the tables, tilings, workspace
// and view subset the batch recorded at bind time.
ltm_status check_current(const ltm_batch* b)
{
    if (!b || !b->bound) return fail(LTM_ERR_WORKSPACE, "batch not bound");
    for (size_t k = 0; k < b->plans.size(); ++k) {
        const ltm_plan* p = b->plans[k];
        if (!p->bound || p->generation != b->gen_bind[k] || p->sub_n != b->sub_bind[k].first ||
            p->sub_i != b->sub_bind[k].second)
            return fail(LTM_ERR_WORKSPACE, "plan " + std::to_string(k) +
                                               " changed (tiling, workspace or view subset) since the "
                                               "batch was bound; create the batch again");
    }
    return LTM_OK;
}

ltm_status run_dir(ltm_batch* b, int d, hipStream_t s)
{
    auto* cams = reinterpret_cast<const BatchCam*>(b->ws + b->cams_off[d]);
    auto* items = reinterpret_cast<const uint32_t*>(b->ws + b->dir[d].items_off);
    auto* ctr = reinterpret_cast<unsigned int*>(b->ws + b->counter_off) + d;
    hipError_t e = hipSuccess;
    if (d == LTM_ADJOINT)
        for (auto* p : b->plans) {
            e = launch_fill64(reinterpret_cast<double*>(p->ws + p->accum_off), p->n_vox, s);
            if (e != hipSuccess) return hip_fail(e, "batch zero accumulators");
        }
    e = launch_batch(cams, items, (uint32_t)b->dir[d].items.size(), ctr, d, b->dir[d].blocks,
                     b->dir[d].lds, s);
    if (e != hipSuccess) return hip_fail(e, "batch sweep");
    if (d == LTM_ADJOINT)
        for (size_t k = 0; k < b->plans.size(); ++k) {
            ltm_plan* p = b->plans[k];
            // the plan's output volume is recorded in its first batch camera
            float* xout = nullptr;
            for (size_t q = 0; q < b->pcs.size(); ++q)
                if (b->pcs[q].first == (int)k) {
                    xout = const_cast<float*>(b->host_cams[LTM_ADJOINT][q].x);
                    break;
                }
            if (!xout) continue;
            e = launch_to_f32(reinterpret_cast<const double*>(p->ws + p->accum_off), xout, p->n_vox, s);
            if (e != hipSuccess) return hip_fail(e, "batch convert");
        }
    return LTM_OK;
}

}  // namespace
}  // namespace ltm

using namespace ltm;

extern "C" {

ltm_status ltm_batch_create(ltm_plan* const* plans, uint32_t n_plans, ltm_batch** out)
{
    if (!out) return fail(LTM_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!plans || n_plans == 0) return fail(LTM_ERR_INVALID, "no plans");
    ltm_batch* b = new (std::nothrow) ltm_batch();
    if (!b) return fail(LTM_ERR_INVALID, "out of host memory");
    for (uint32_t i = 0; i < n_plans; ++i) {
        if (!plans[i] || !plans[i]->bound) {
            delete b;
            return fail(LTM_ERR_WORKSPACE, "plan " + std::to_string(i) + " is null or unbound");
        }
        b->plans.push_back(plans[i]);
        b->gen_create.push_back(plans[i]->generation);
        for (size_t c = 0; c < plans[i]->cams.size(); ++c) b->pcs.push_back({(int)i, (int)c});
    }
    if (b->pcs.size() >= (1u << (32 - kTileBits))) {
        delete b;
        return fail(LTM_ERR_INVALID, "too many cameras in one batch");
    }
    uint64_t off = 0;
    for (int d = 0; d < 2; ++d) {
        std::vector<std::pair<double, uint32_t>> order;   // (cost per tile, batch camera)
        size_t lds = 0;
        for (size_t q = 0; q < b->pcs.size(); ++q) {
            const ltm_plan* p = b->plans[b->pcs[q].first];
            const CamDev dv = bound_dev(p, p->cams[b->pcs[q].second], d);
            if ((uint64_t)dv.n_tiles >= (1ull << kTileBits)) {
                delete b;
                return fail(LTM_ERR_INVALID, "a camera has more than 2^20 tiles");
            }
            order.push_back({(double)dv.items_per_split * dv.ru * dv.rv * dv.S, (uint32_t)q});
            lds = std::max(lds, march_lds_bytes(dv, d));
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const auto& a, const auto& c) { return a.first > c.first; });
        for (auto& o : order) {
            const ltm_plan* p = b->plans[b->pcs[o.second].first];
            const CamDev dv = bound_dev(p, p->cams[b->pcs[o.second].second], d);
            for (int t = 0; t < dv.n_tiles; ++t) b->dir[d].items.push_back((o.second << kTileBits) | (uint32_t)t);
        }
        b->dir[d].lds = lds;
        b->cams_off[d] = off;
        off = align256(off + sizeof(BatchCam) * b->pcs.size());
        b->dir[d].items_off = off;
        off = align256(off + 4 * b->dir[d].items.size());
    }
    b->counter_off = off;
    b->ws_bytes = off + 256;
    clear_error();
    *out = b;
    return LTM_OK;
}

void ltm_batch_destroy(ltm_batch* b)
{
    if (!b) return;
    release_graph(b);
    delete b;
}

ltm_status ltm_batch_workspace_bytes(const ltm_batch* b, uint64_t* bytes)
{
    if (!b || !bytes) return fail(LTM_ERR_INVALID, "null argument");
    *bytes = b->ws_bytes;
    return LTM_OK;
}

ltm_status ltm_batch_bind(ltm_batch* b, void* ws, uint64_t bytes, const float* const* x_in,
                          float* const* y, float* const* x_out, void* stream)
{
    if (!b || !x_in || !y || !x_out) return fail(LTM_ERR_INVALID, "null argument");
    if (!ws || bytes < b->ws_bytes)
        return fail(LTM_ERR_WORKSPACE, "batch workspace of " + std::to_string(b->ws_bytes) +
                                           " bytes required");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(LTM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    for (size_t k = 0; k < b->plans.size(); ++k)
        if (!x_in[k] || !y[k] || !x_out[k]) return fail(LTM_ERR_INVALID, "null buffer for plan " + std::to_string(k));
    // the work lists and LDS sizes were built from the plans at creation
    for (size_t k = 0; k < b->plans.size(); ++k)
        if (!b->plans[k]->bound || b->plans[k]->generation != b->gen_create[k])
            return fail(LTM_ERR_WORKSPACE, "plan " + std::to_string(k) +
                                               " changed (tiling or workspace) since the batch was "
                                               "created; create the batch again");
    release_graph(b);
    b->bound = false;
    b->ws = static_cast<char*>(ws);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int d = 0; d < 2; ++d) {
        b->host_cams[d].clear();
        for (auto& pc : b->pcs) {
            const ltm_plan* p = b->plans[pc.first];
            BatchCam bc;
            bc.cam = bound_dev(p, p->cams[pc.second], d);
            bc.x = d == LTM_FORWARD ? x_in[pc.first] : x_out[pc.first];
            bc.y = y[pc.first];
            bc.xacc = reinterpret_cast<double*>(p->ws + p->accum_off);
            b->host_cams[d].push_back(bc);
        }
        b->dir[d].blocks = cus * batch_blocks_per_cu(d, b->dir[d].lds);
        e = hipMemcpyAsync(b->ws + b->cams_off[d], b->host_cams[d].data(),
                           sizeof(BatchCam) * b->host_cams[d].size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->ws + b->dir[d].items_off, b->dir[d].items.data(),
                               4 * b->dir[d].items.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "batch upload");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    b->gen_bind.clear();
    b->sub_bind.clear();
    for (auto* p : b->plans) {
        b->gen_bind.push_back(p->generation);
        b->sub_bind.push_back({p->sub_n, p->sub_i});
    }
    b->bound = true;
    clear_error();
    return LTM_OK;
}

ltm_status ltm_batch_project(ltm_batch* b, void* stream)
{
    ltm_status st = check_current(b);
    if (st != LTM_OK) return st;
    return run_dir(b, LTM_FORWARD, static_cast<hipStream_t>(stream));
}

ltm_status ltm_batch_backproject(ltm_batch* b, void* stream)
{
    ltm_status st = check_current(b);
    if (st != LTM_OK) return st;
    return run_dir(b, LTM_ADJOINT, static_cast<hipStream_t>(stream));
}

ltm_status ltm_batch_sweep(ltm_batch* b, void* stream)
{
    ltm_status st = ltm_batch_project(b, stream);
    if (st == LTM_OK) st = ltm_batch_backproject(b, stream);
    return st;
}

ltm_status ltm_batch_graph_capture(ltm_batch* b, void* stream)
{
    ltm_status cur = check_current(b);
    if (cur != LTM_OK) return cur;
    if (!stream) return fail(LTM_ERR_INVALID, "graph capture needs a non-null stream");
    hipStream_t s = static_cast<hipStream_t>(stream);
    release_graph(b);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    ltm_status st = ltm_batch_sweep(b, stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st != LTM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        release_graph(b);
        return hip_fail(e, "instantiate graph");
    }
    return LTM_OK;
}

ltm_status ltm_batch_graph_launch(ltm_batch* b, void* stream)
{
    if (!b || !b->exec) return fail(LTM_ERR_INVALID, "no captured graph");
    ltm_status cur = check_current(b);
    if (cur != LTM_OK) return cur;
    hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return LTM_OK;
}

}  // extern "C"
