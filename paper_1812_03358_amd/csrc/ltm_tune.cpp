// Tilings chosen by measurement.  A tiling changes only how a camera's rays
// are grouped into workgroups, staged and summed, never which samples are
// taken, so the tuner may pick any tiling whose output matches the current
// one: each candidate runs on a one-camera copy of the plan, is rejected
// unless its output is within relative L2 1e-6 of the current tiling's (the
// FP64 sums only change order), and is timed with HIP events.  The search
// has two stages: tile shape, lane order, slab depth and brick size at full
// occupancy, then the occupancy cap (workgroups per CU) for the three fastest
// shapes.  Results are cached in a text file keyed by the GPU architecture,
// the grid and the camera descriptor.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "ltm_internal.h"

namespace ltm {
namespace {

constexpr double kParity = 1e-6;
constexpr int kOccupancyShapes = 3;
const uint32_t kOccupancyCaps[] = {2, 3};

uint64_t align256(uint64_t v) { return (v + 255u) & ~uint64_t(255u); }

uint64_t fnv1a(const void* p, size_t n, uint64_t h)
{
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string cache_key(const std::string& arch, const ltm_grid& g, const ltm_camera& c, int dir)
{
    uint64_t h = fnv1a(&g, sizeof(g), 1469598103934665603ull);
    h = fnv1a(&c, sizeof(c), h);
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|%s|kind%u|grid%ux%ux%u|det%ux%u|mla%ux%u|R%ux%u|S%u|%016llx",
                  arch.c_str(), dir == LTM_FORWARD ? "A" : "AT", c.kind, g.nx, g.ny, g.nz, c.det_nu,
                  c.det_nv, c.mla_nu, c.mla_nv, c.rays_u, c.rays_v, c.samples,
                  (unsigned long long)h);
    return buf;
}

std::string tiling_text(const ltm_tiling& t)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%u %u %u %u %u %u %u %u %.17g", t.tile_u, t.tile_v, t.block_u,
                  t.block_v, t.order, t.splits, t.brick_floats, t.groups_per_cu, t.chunk_mm);
    return buf;
}

bool parse_tiling(const std::string& s, ltm_tiling& t)
{
    std::istringstream in(s);
    t = ltm_tiling{};
    in >> t.tile_u >> t.tile_v >> t.block_u >> t.block_v >> t.order >> t.splits >> t.brick_floats >>
        t.groups_per_cu >> t.chunk_mm;
    return !in.fail();
}

// cache file: one line per key, "key<TAB>tiling<TAB>ms default_ms"
struct CacheEntry {
    std::string tiling;
    std::string times;
};

std::map<std::string, CacheEntry> read_cache(const char* path)
{
    std::map<std::string, CacheEntry> m;
    if (!path || !*path) return m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        const size_t a = line.find('\t');
        const size_t b = a == std::string::npos ? a : line.find('\t', a + 1);
        if (b == std::string::npos) continue;
        m[line.substr(0, a)] = {line.substr(a + 1, b - a - 1), line.substr(b + 1)};
    }
    return m;
}

bool write_cache(const char* path, const std::map<std::string, CacheEntry>& m)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return false;
        f << "# libltm tilings: key\ttile_u tile_v block_u block_v order splits brick_floats "
             "groups_per_cu chunk_mm\tms default_ms\n";
        for (const auto& kv : m) f << kv.first << '\t' << kv.second.tiling << '\t' << kv.second.times << '\n';
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

// Rays a pixel visits (hexagonal cameras: 3 x 3 lenslets).
uint32_t rays_of(const ltm_camera& c)
{
    return c.rays_u * c.rays_v * (c.kind == LTM_PLENOPTIC_HEX ? 9u : 1u);
}

// Stage-1 candidates: tile shape, lane order flags, slab depth and brick.
std::vector<ltm_tiling> shape_candidates(const ltm_grid& g, const ltm_camera& c, int dir)
{
    std::vector<ltm_tiling> out;
    const bool pl = c.kind == LTM_PLENOPTIC;
    const uint64_t k = pl ? (uint64_t)(c.det_nu / c.mla_nu) * (c.det_nv / c.mla_nv) : 1;
    const uint64_t R = rays_of(c);
    auto push = [&](uint32_t t, uint32_t blk, uint32_t order, uint32_t splits, uint32_t brick,
                    double chunk) {
        ltm_tiling x{};
        x.tile_u = x.tile_v = t;
        x.block_u = x.block_v = blk;
        x.order = order;
        x.splits = splits;
        x.brick_floats = brick;
        x.chunk_mm = chunk * g.pitch_mm;
        if (check_tiling(g, c, x) != LTM_OK) return;
        for (const ltm_tiling& y : out)
            if (std::memcmp(&x, &y, sizeof(x)) == 0) return;    // two group sizes gave one split
        out.push_back(x);
    };
    if (dir == LTM_FORWARD) {
        const std::vector<uint32_t> tiles = pl ? std::vector<uint32_t>{1, 2} : std::vector<uint32_t>{1};
        const std::vector<uint32_t> blocks = pl ? std::vector<uint32_t>{16} : std::vector<uint32_t>{16, 8};
        for (uint32_t t : tiles)
            for (uint32_t blk : blocks) {
                const uint64_t items = (uint64_t)t * t * (pl ? k : (uint64_t)blk * blk);
                for (uint32_t splits : {1u, 4u}) {
                    if (items % splits || items / splits > 2048 || items / splits * R > 8192) continue;
                    for (uint32_t order : {0u, 2u})
                        for (double chunk : {16.0, 32.0, 64.0})
                            for (uint32_t brick : {4096u, 6144u, 8192u}) push(t, blk, order, splits, brick, chunk);
                }
            }
    } else {
        const std::vector<uint32_t> tiles = pl ? std::vector<uint32_t>{2, 4} : std::vector<uint32_t>{1, 2};
        const std::vector<uint32_t> blocks = pl ? std::vector<uint32_t>{16} : std::vector<uint32_t>{8, 16};
        for (uint32_t t : tiles)
            for (uint32_t blk : blocks) {
                const uint64_t items = (uint64_t)t * t * (pl ? k : (uint64_t)blk * blk);
                for (uint64_t per : {64ull, 256ull}) {
                    const uint64_t splits = std::max<uint64_t>(1, items / per);
                    if (items % splits || items / splits > 2048 || items / splits * R > 8192) continue;
                    // bits: 0 lanes across lenslets, 1 no rotation, 3 staggered walks,
                    // 4 merged cells, 5 plane windows, 6 even stagger offsets
                    for (uint32_t order : {26u, 27u, 40u, 41u, 42u, 43u, 104u, 105u, 106u, 107u})
                        for (double chunk : {16.0, 32.0})
                            for (uint32_t brick : {8192u, 12288u})
                                push(t, blk, order, (uint32_t)splits, brick, chunk);
                }
            }
    }
    clear_error();
    return out;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// One camera of a plan on the tuner's workspace: a one-camera plan whose
// tiling of `dir` is set and bound on demand, its input and output buffers.
struct Bench {
    ltm_plan* sub = nullptr;
    int dir = 0;
    const float* in = nullptr;
    float* out = nullptr;
    float* ref = nullptr;
    double* sums = nullptr;
    uint64_t n_out = 0;
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    hipStream_t s = nullptr;
    Timer tm;
    ~Bench() { ltm_plan_destroy(sub); }

    ltm_status apply(const ltm_tiling& t)
    {
        ltm_status st = ltm_plan_set_tiling(sub, (uint32_t)dir, 0, &t);
        if (st != LTM_OK) return st;
        uint64_t need = 0;
        ltm_plan_workspace_bytes(sub, &need);
        if (need > ws_bytes) return fail(LTM_ERR_WORKSPACE, "candidate tables exceed the tuner's workspace");
        return ltm_plan_bind_workspace(sub, ws, ws_bytes, s);
    }
    ltm_status run(float* dst)
    {
        return dir == LTM_FORWARD ? ltm_project(sub, in, dst, s) : ltm_backproject(sub, in, dst, s);
    }
    // median of `reps` event-timed runs after one untimed run
    ltm_status time(uint32_t reps, double& ms)
    {
        ltm_status st = run(out);
        if (st != LTM_OK) return st;
        std::vector<float> t;
        for (uint32_t r = 0; r < reps; ++r) {
            hipError_t e = hipEventRecord(tm.a, s);
            if (e == hipSuccess) {
                st = run(out);
                if (st != LTM_OK) return st;
                e = hipEventRecord(tm.b, s);
            }
            if (e == hipSuccess) e = hipEventSynchronize(tm.b);
            float v = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&v, tm.a, tm.b);
            if (e != hipSuccess) return hip_fail(e, "autotune timing");
            t.push_back(v);
        }
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return LTM_OK;
    }
    // relative L2 distance of `out` from `ref`
    ltm_status error(double& err)
    {
        hipError_t e = launch_diff_sumsq(out, ref, n_out, sums, s);
        double h[2] = {0.0, 0.0};
        if (e == hipSuccess) e = hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "autotune parity");
        err = std::sqrt(h[0]) / (h[1] > 0.0 ? std::sqrt(h[1]) : 1.0);
        if (!std::isfinite(err)) err = INFINITY;
        return LTM_OK;
    }
};

// Workspace one camera's tuning needs: a one-camera plan's tables for the
// largest candidate of each direction (the two directions' tables add up,
// and a direction's size does not depend on the other's tiling), plus two
// outputs and the parity sums.
ltm_status camera_bytes(const ltm_plan* p, uint32_t ci, uint64_t& tables, uint64_t& outputs)
{
    const CamHost& c = p->cams[ci];
    ltm_plan* sub = nullptr;
    ltm_status st = ltm_plan_create(&p->grid, &c.desc, 1, &sub);
    if (st != LTM_OK) return st;
    ltm_tiling worst[2] = {c.tiling[0], c.tiling[1]};
    for (int dir = 0; dir < 2; ++dir) {
        ltm_tiling other = c.tiling[1 - dir];
        ltm_plan_set_tiling(sub, (uint32_t)(1 - dir), 0, &other);
        std::vector<ltm_tiling> cands = shape_candidates(p->grid, c.desc, dir);
        cands.push_back(c.tiling[dir]);
        uint64_t most = 0;
        for (const ltm_tiling& t : cands) {
            if (ltm_plan_set_tiling(sub, (uint32_t)dir, 0, &t) != LTM_OK) continue;
            uint64_t b = 0;
            ltm_plan_workspace_bytes(sub, &b);
            if (b > most) {
                most = b;
                worst[dir] = t;
            }
        }
    }
    st = ltm_plan_set_tiling(sub, 0, 0, &worst[0]);
    if (st == LTM_OK) st = ltm_plan_set_tiling(sub, 1, 0, &worst[1]);
    if (st == LTM_OK) st = ltm_plan_workspace_bytes(sub, &tables);
    ltm_plan_destroy(sub);
    if (st != LTM_OK) return st;
    clear_error();
    outputs = 2 * align256(4 * std::max<uint64_t>(p->n_vox, c.npix)) + 256;
    return LTM_OK;
}

}  // namespace
}  // namespace ltm

using namespace ltm;

extern "C" {

ltm_status ltm_autotune_candidates(const ltm_plan* p, uint32_t dir, uint32_t cam, ltm_tiling* out,
                                   uint32_t capacity, uint32_t* count)
{
    if (!p || !count) return fail(LTM_ERR_INVALID, "null argument");
    if (dir > 1 || cam >= p->cams.size()) return fail(LTM_ERR_INVALID, "bad direction or camera");
    std::vector<ltm_tiling> c = shape_candidates(p->grid, p->cams[cam].desc, (int)dir);
    *count = (uint32_t)c.size();
    if (out)
        for (uint32_t i = 0; i < std::min<uint32_t>(capacity, (uint32_t)c.size()); ++i) out[i] = c[i];
    return LTM_OK;
}

ltm_status ltm_autotune_workspace_bytes(const ltm_plan* p, uint64_t* bytes)
{
    if (!p || !bytes) return fail(LTM_ERR_INVALID, "null argument");
    uint64_t best = 0;
    for (uint32_t ci = 0; ci < p->cams.size(); ++ci) {
        uint64_t tables = 0, outputs = 0;
        ltm_status st = camera_bytes(p, ci, tables, outputs);
        if (st != LTM_OK) return st;
        best = std::max(best, align256(tables) + outputs);
    }
    *bytes = best;
    return LTM_OK;
}

ltm_status ltm_autotune(ltm_plan* p, const float* x, const float* y, void* ws, uint64_t bytes,
                        const char* cache_path, uint32_t reps, double* ms, void* stream)
{
    if (!p || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (reps == 0) return fail(LTM_ERR_INVALID, "reps must be at least 1");
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(LTM_ERR_WORKSPACE, "autotune workspace missing or not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::string arch = arch_name();
    std::map<std::string, CacheEntry> cache = read_cache(cache_path);
    bool cache_dirty = false;
    for (uint32_t ci = 0; ci < p->cams.size(); ++ci) {
        CamHost& c = p->cams[ci];
        uint64_t tables = 0, outputs = 0;
        ltm_status st = camera_bytes(p, ci, tables, outputs);
        if (st != LTM_OK) return st;
        tables = align256(tables);
        if (bytes < tables + outputs)
            return fail(LTM_ERR_WORKSPACE, "autotune workspace of " + std::to_string(tables + outputs) +
                                               " bytes required");
        for (int dir = 0; dir < 2; ++dir) {
            Bench b;
            st = ltm_plan_create(&p->grid, &c.desc, 1, &b.sub);
            if (st != LTM_OK) return st;
            b.dir = dir;
            b.s = s;
            b.ws = static_cast<char*>(ws);
            b.ws_bytes = tables;
            b.n_out = dir == LTM_FORWARD ? c.npix : p->n_vox;
            char* o = b.ws + tables;
            b.out = reinterpret_cast<float*>(o);
            b.ref = reinterpret_cast<float*>(o + align256(4 * std::max<uint64_t>(p->n_vox, c.npix)));
            b.sums = reinterpret_cast<double*>(o + 2 * align256(4 * std::max<uint64_t>(p->n_vox, c.npix)));
            b.in = dir == LTM_FORWARD ? x : y + c.y_off;
            if (hipEventCreate(&b.tm.a) != hipSuccess || hipEventCreate(&b.tm.b) != hipSuccess)
                return fail(LTM_ERR_DEVICE, "autotune events");
            ltm_tiling other = c.tiling[1 - dir];
            if ((st = ltm_plan_set_tiling(b.sub, (uint32_t)(1 - dir), 0, &other)) != LTM_OK) return st;
            // reference: the camera's current tiling (as adapted at bind)
            const ltm_tiling current = c.tiling[dir];
            if ((st = b.apply(current)) != LTM_OK) return st;
            double default_ms = 0.0;
            if ((st = b.time(reps, default_ms)) != LTM_OK) return st;
            hipError_t e = hipMemcpyAsync(b.ref, b.out, 4 * b.n_out, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "autotune reference copy");
            double best_ms = default_ms;
            ltm_tiling best = current;
            // every candidate passes the parity gate before it is timed
            auto consider = [&](const ltm_tiling& t, double& t_ms) -> ltm_status {
                t_ms = INFINITY;
                if (check_tiling(p->grid, c.desc, t) != LTM_OK) {
                    clear_error();
                    return LTM_OK;
                }
                ltm_status r = b.apply(t);
                if (r == LTM_ERR_WORKSPACE || r == LTM_ERR_INVALID) {
                    clear_error();
                    return LTM_OK;
                }
                if (r != LTM_OK) return r;
                if ((r = b.run(b.out)) != LTM_OK) return r;
                double err = 0.0;
                if ((r = b.error(err)) != LTM_OK) return r;
                if (!(err <= kParity)) return LTM_OK;
                if ((r = b.time(reps, t_ms)) != LTM_OK) return r;
                if (t_ms < best_ms) {
                    best_ms = t_ms;
                    best = t;
                }
                return LTM_OK;
            };
            const std::string key = cache_key(arch, p->grid, c.desc, dir);
            auto hit = cache.find(key);
            ltm_tiling cached{};
            double t_ms = 0.0;
            if (hit != cache.end() && parse_tiling(hit->second.tiling, cached)) {
                if ((st = consider(cached, t_ms)) != LTM_OK) return st;
            } else {
                std::vector<std::pair<double, ltm_tiling>> timed;
                for (const ltm_tiling& t : shape_candidates(p->grid, c.desc, dir)) {
                    if ((st = consider(t, t_ms)) != LTM_OK) return st;
                    if (std::isfinite(t_ms)) timed.push_back({t_ms, t});
                }
                timed.push_back({default_ms, current});
                std::sort(timed.begin(), timed.end(),
                          [](const std::pair<double, ltm_tiling>& a, const std::pair<double, ltm_tiling>& b2) {
                              return a.first < b2.first;
                          });
                for (size_t i = 0; i < timed.size() && i < (size_t)kOccupancyShapes; ++i)
                    for (uint32_t cap : kOccupancyCaps) {
                        ltm_tiling t = timed[i].second;
                        if (t.groups_per_cu == cap) continue;
                        t.groups_per_cu = cap;
                        if ((st = consider(t, t_ms)) != LTM_OK) return st;
                    }
                if (cache_path && *cache_path) {
                    char buf[64];
                    std::snprintf(buf, sizeof(buf), "%.5f %.5f", best_ms, default_ms);
                    cache[key] = {tiling_text(best), buf};
                    cache_dirty = true;
                }
            }
            if (ms) {
                ms[4 * ci + 2 * dir] = best_ms;
                ms[4 * ci + 2 * dir + 1] = default_ms;
            }
            const ltm_tiling& now = c.tiling[dir];
            if (std::memcmp(&best, &now, sizeof(best)) != 0) {
                if ((st = ltm_plan_set_tiling(p, (uint32_t)dir, ci, &best)) != LTM_OK) return st;
            }
        }
    }
    if (cache_dirty && !write_cache(cache_path, cache))
        return fail(LTM_ERR_INVALID, std::string("cannot write the tiling cache ") + cache_path);
    clear_error();
    return LTM_OK;
}

}  // extern "C"
