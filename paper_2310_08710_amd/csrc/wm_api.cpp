// wm_api.cpp -- the C ABI declared in include/wm.h: argument validation,
// workspace carving, launch configuration, the rollout autotuner and error
// reporting.  Validation never touches the device: every check below runs on
// host-visible values before the first launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/wm.h"
#include "wm_internal.h"

namespace {

thread_local std::string g_msg;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_msg = buf;
    return code;
}

int ok()
{
    g_msg.clear();
    return WM_OK;
}

int device_status(const char *where)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(WM_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
    return ok();
}

#define CHECK(expr)                   \
    do {                              \
        const int _rc = (expr);       \
        if (_rc != WM_OK)             \
            return _rc;               \
    } while (0)

int check_batch(const wm_batch *b)
{
    if (!b)
        return fail(WM_ERR_NULL, "batch is NULL");
    if (!b->obj_off || !b->rg_off)
        return fail(WM_ERR_NULL, "batch offsets are NULL");
    if (b->num_scenarios < 1)
        return fail(WM_ERR_RANGE, "num_scenarios = %d < 1", b->num_scenarios);
    if (b->total_objects < 0 || b->total_rg_points < 0 || b->max_objects < 0 || b->max_rg_points < 0)
        return fail(WM_ERR_SHAPE, "negative batch size");
    if (b->max_objects > b->total_objects || b->max_rg_points > b->total_rg_points)
        return fail(WM_ERR_SHAPE, "max_objects/max_rg_points exceed the totals");
    if (b->max_objects > WM_MAX_OBJECTS)
        return fail(WM_ERR_UNSUPPORTED, "max_objects = %d > %d", b->max_objects, WM_MAX_OBJECTS);
    return WM_OK;
}

int check_state(const wm_state *s, const char *name)
{
    if (!s)
        return fail(WM_ERR_NULL, "%s is NULL", name);
    if (!s->x || !s->y || !s->yaw || !s->vx || !s->vy || !s->length || !s->width || !s->valid)
        return fail(WM_ERR_NULL, "%s has a NULL member", name);
    return WM_OK;
}

int check_rg(const wm_roadgraph *r)
{
    if (!r->x || !r->y || !r->dir_x || !r->dir_y || !r->type || !r->valid)
        return fail(WM_ERR_NULL, "roadgraph has a NULL member");
    return WM_OK;
}

int check_dt(float dt)
{
    if (!(dt > 0.f) || !std::isfinite(dt))
        return fail(WM_ERR_RANGE, "dt = %g must be finite and > 0", (double)dt);
    return WM_OK;
}

int check_ws(const void *ws, size_t have, size_t need)
{
    if (need == 0)
        return WM_OK;
    if (!ws)
        return fail(WM_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (have < need)
        return fail(WM_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", have, need);
    return WM_OK;
}

struct Tune {
    int G, CW;
};

std::mutex g_tune_mu;
std::map<std::pair<int, int>, Tune> g_tune_table;

// Tunings kept across processes: with WM_TUNE_CACHE naming a file, every
// tuning wm_autotune picks is appended to it as a line
//   wm-tune <version> <arch> <compute units> <object bucket> <point bucket> <unit_objects> <edge_splits>
// and a later process takes the last matching line instead of timing again
// (wm_autotune) or of the default (a NULL tuning).  The version changes with
// the rollout kernel's work layout, so that older lines stop matching.
constexpr int kTuneCacheVersion = 3;

std::string tune_device_tag()
{
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos)
            arch = arch.substr(0, colon);   // gfx950, without the feature flags
    }
    return arch + " " + std::to_string(cus);
}

// The cached tuning of bucket `key` on this device, from the file WM_TUNE_CACHE.
bool tune_cache_lookup(std::pair<int, int> key, Tune *out)
{
    const char *path = std::getenv("WM_TUNE_CACHE");
    if (!path || !*path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    const std::string dev = tune_device_tag();
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char arch[64];
        int ver = 0, cus = 0, ob = 0, pb = 0, U = 0, G = 0;
        if (std::sscanf(line, "wm-tune %d %63s %d %d %d %d %d", &ver, arch, &cus, &ob, &pb, &U, &G) != 7)
            continue;
        if (ver != kTuneCacheVersion || std::string(arch) + " " + std::to_string(cus) != dev ||
            ob != key.first || pb != key.second)
            continue;
        if ((U != 64 && U != 128 && U != 256) || (G != 1 && G != 2 && G != 4 && G != 8 && G != 16) || U * G > 512)
            continue;
        *out = Tune{G, U / 64};   // the last matching line wins
        found = true;
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(std::pair<int, int> key, const wm_tuning &t)
{
    const char *path = std::getenv("WM_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f, "wm-tune %d %s %d %d %d %d\n", kTuneCacheVersion, tune_device_tag().c_str(), key.first,
                 key.second, t.unit_objects, t.edge_splits);
    std::fclose(f);
}

std::pair<int, int> tune_key(const wm_batch *b)
{
    int ob = 0, pb = 0;
    while ((1 << ob) < b->max_objects)
        ++ob;
    while ((1 << pb) < b->max_rg_points)
        ++pb;
    return {ob, pb};
}

// max_threads is the work-group size limit of the kernel the tuning is for.
int resolve_tune(const wm_batch *b, const wm_tuning *t, int max_threads, Tune *out)
{
    if (t) {
        const int U = t->unit_objects, G = t->edge_splits;
        if (U != 64 && U != 128 && U != 256)
            return fail(WM_ERR_RANGE, "unit_objects = %d not in {64, 128, 256}", U);
        if (G != 1 && G != 2 && G != 4 && G != 8 && G != 16)
            return fail(WM_ERR_RANGE, "edge_splits = %d not in {1, 2, 4, 8, 16}", G);
        if (U * G > max_threads)
            return fail(WM_ERR_RANGE, "unit_objects * edge_splits = %d > %d", U * G, max_threads);
        out->G = G;
        out->CW = U / 64;
        return WM_OK;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const std::pair<int, int> key = tune_key(b);
    auto it = g_tune_table.find(key);
    if (it != g_tune_table.end()) {
        *out = it->second;
    } else {
        if (!tune_cache_lookup(key, out)) {
            out->G = 8;
            out->CW = 1;
        }
        g_tune_table[key] = *out;   // the cache file is read once per bucket
    }
    return WM_OK;
}

size_t workspace_bytes(const wm_batch *b, int T, int K)
{
    return wm::ws_layout(b->num_scenarios, b->total_objects, b->total_rg_points, T, K).total;
}

// ---- kernel timing (profiling aid) ----
constexpr int kProfKinds = 4;
constexpr size_t kProfMax = 4096;
struct ProfState {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> used[kProfKinds];
    std::vector<hipEvent_t> pool;   // reused; never destroyed (no HIP calls at thread or process exit)
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        return e;
    }
};
// process-wide: autograd runs backward passes on its own threads
ProfState g_prof;
std::mutex g_prof_mu;

// Brackets one launch with events when profiling is on.
struct ProfScope {
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int k, hipStream_t s) : kind(k), st(s)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (g_prof.on && g_prof.used[kind].size() < kProfMax) {
            a = g_prof.get();
            b = g_prof.get();
            if (a && b)
                (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope()
    {
        if (a && b) {
            (void)hipEventRecord(b, st);
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof.used[kind].emplace_back(a, b);
        }
    }
};

} // namespace

extern "C" {

size_t wm_workspace_bytes(const wm_batch *batch, int32_t T, int32_t ckpt_every)
{
    if (check_batch(batch) != WM_OK || T < 0 || ckpt_every < 0)
        return 0;
    return workspace_bytes(batch, T, ckpt_every);
}

size_t wm_rollout_workspace_bytes(const wm_batch *batch, int32_t T, int32_t ckpt_every)
{
    return wm_workspace_bytes(batch, T, ckpt_every);
}

const char *wm_error_string(int code)
{
    switch (code) {
    case WM_OK: return "ok";
    case WM_ERR_NULL: return "a required pointer is NULL";
    case WM_ERR_RANGE: return "a scalar argument is out of range";
    case WM_ERR_SHAPE: return "inconsistent sizes";
    case WM_ERR_WORKSPACE: return "workspace missing or too small";
    case WM_ERR_UNSUPPORTED: return "size not supported by the kernels";
    case WM_ERR_DEVICE: return "HIP runtime error";
    default: return "unknown error code";
    }
}

const char *wm_last_error_message(void) { return g_msg.c_str(); }

int wm_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.on = on != 0;
    return ok();
}

int wm_profile_collect(int which, float *total_ms, int32_t *launches)
{
    if (which < 0 || which >= kProfKinds)
        return fail(WM_ERR_RANGE, "profile kind %d out of range", which);
    if (!total_ms || !launches)
        return fail(WM_ERR_NULL, "total_ms or launches is NULL");
    float tot = 0.f;
    int cnt = 0;
    int rc = WM_OK;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &p : g_prof.used[which]) {
        float ms = 0.f;
        if (rc == WM_OK) {
            hipError_t e = hipEventSynchronize(p.second);
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, p.first, p.second);
            if (e != hipSuccess)
                rc = fail(WM_ERR_DEVICE, "wm_profile_collect: %s", hipGetErrorString(e));
            tot += ms;
            ++cnt;
        }
        g_prof.pool.push_back(p.first);
        g_prof.pool.push_back(p.second);
    }
    g_prof.used[which].clear();
    *total_ms = tot;
    *launches = cnt;
    return rc == WM_OK ? ok() : rc;
}

enum class StepWs { Given, Prepared, Scratch };

// `Prepared`: the workspace already holds this road graph's compacted edges
// (wm_roadgraph_prepare), so the compaction is skipped.  `Scratch`: the
// workspace is the device's WM_NOALLOC_SCRATCH_BYTES array (ws is ignored).
static int step_impl(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
                     const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *m, void *ws, size_t ws_bytes,
                     void *stream, StepWs wsk)
{
    const bool prepared = wsk == StepWs::Prepared;
    const char *name = wsk == StepWs::Given ? "wm_step" : prepared ? "wm_step_prepared" : "wm_step_noalloc";
    CHECK(check_batch(batch));
    CHECK(check_state(cur, "cur"));
    CHECK(check_state(log_next, "log_next"));
    CHECK(check_state(next, "next"));
    if (!act || !act->accel || !act->curvature || !act->controlled)
        return fail(WM_ERR_NULL, "action is NULL or has a NULL member");
    CHECK(check_dt(dt));
    if (next->x == cur->x)
        return fail(WM_ERR_RANGE, "next must not alias cur");
    const bool want_off = m && rg && (m->offroad || m->offroad_margin);
    if (want_off)
        CHECK(check_rg(rg));
    if (m && m->reward && (!m->collision || (rg && !m->offroad)))
        return fail(WM_ERR_NULL, "reward needs the collision (and, with a road graph, offroad) outputs");
    const wm::WsLayout L = wm::ws_layout(batch->num_scenarios, batch->total_objects, batch->total_rg_points, 0, 0);
    if (want_off && wsk == StepWs::Scratch && L.total > WM_NOALLOC_SCRATCH_BYTES)
        return fail(WM_ERR_UNSUPPORTED,
                    "wm_step_noalloc: off-road metrics of this batch (%d scenarios, %d road points) need %zu bytes "
                    "of workspace, more than the %zu of the device scratch; use wm_step with a workspace",
                    batch->num_scenarios, batch->total_rg_points, L.total, (size_t)WM_NOALLOC_SCRATCH_BYTES);
    if (want_off && wsk == StepWs::Scratch) {
        unsigned char *p = nullptr;
        const hipError_t e = wm::noalloc_scratch(&p);
        if (e != hipSuccess)
            return fail(WM_ERR_DEVICE, "wm_step_noalloc: device scratch address: %s", hipGetErrorString(e));
        ws = p;
        ws_bytes = WM_NOALLOC_SCRATCH_BYTES;
    }
    if (want_off)
        CHECK(check_ws(ws, ws_bytes, L.total));
    hipStream_t st = (hipStream_t)stream;
    wm::StepArgs a{batch->obj_off, *cur, *act, *log_next, *next, dt, m ? m->log_div : nullptr,
                   m ? m->infeasible : nullptr};
    wm::launch_dynamics(*batch, a, st);
    if (m && (m->collision || m->overlap_margin)) {
        wm::OverlapArgs o{batch->obj_off, *next, nullptr, nullptr, nullptr, m->collision, m->overlap_margin,
                          batch->max_objects, 64};
        wm::launch_overlap(*batch, o, st);
    }
    if (want_off) {
        unsigned char *w = (unsigned char *)ws;
        Tune tn;
        CHECK(resolve_tune(batch, nullptr, 1024, &tn));
        tn.CW = 1;
        if (tn.G > 16)
            tn.G = 16;
        if (!prepared) {
            wm::launch_compact_edges(*batch, *rg, w, L, st);
            wm::launch_edge_boxes(*batch, w, L, st);
        }
        wm::OffroadArgs o{batch->obj_off, batch->rg_off, *next, wm::ws_edges(w, L), m->offroad, m->offroad_margin,
                          nullptr, tn.G, tn.CW};
        wm::launch_offroad(*batch, o, st);
    }
    if (m && m->reward)
        wm::launch_reward(*batch, m->collision, rg ? m->offroad : nullptr, m->reward, st);
    return device_status(name);
}

int wm_step(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
            const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *m, void *ws, size_t ws_bytes,
            void *stream)
{
    return step_impl(batch, cur, act, log_next, rg, dt, next, m, ws, ws_bytes, stream, StepWs::Given);
}

int wm_step_prepared(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
                     const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *m, void *ws, size_t ws_bytes,
                     void *stream)
{
    return step_impl(batch, cur, act, log_next, rg, dt, next, m, ws, ws_bytes, stream, StepWs::Prepared);
}

int wm_step_noalloc(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
                    const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *m, void *stream)
{
    return step_impl(batch, cur, act, log_next, rg, dt, next, m, nullptr, 0, stream, StepWs::Scratch);
}

int wm_roadgraph_prepare(const wm_batch *batch, const wm_roadgraph *rg, void *ws, size_t ws_bytes, void *stream)
{
    CHECK(check_batch(batch));
    if (!rg)
        return fail(WM_ERR_NULL, "roadgraph is NULL");
    CHECK(check_rg(rg));
    const wm::WsLayout L = wm::ws_layout(batch->num_scenarios, batch->total_objects, batch->total_rg_points, 0, 0);
    CHECK(check_ws(ws, ws_bytes, L.total));
    wm::launch_compact_edges(*batch, *rg, (unsigned char *)ws, L, (hipStream_t)stream);
    wm::launch_edge_boxes(*batch, (unsigned char *)ws, L, (hipStream_t)stream);
    return device_status("wm_roadgraph_prepare");
}

int wm_inverse_action(const wm_batch *batch, const wm_state *cur, const wm_state *next, float dt, float *accel,
                      float *curvature, uint8_t *valid_out, void *stream)
{
    CHECK(check_batch(batch));
    CHECK(check_state(cur, "cur"));
    CHECK(check_state(next, "next"));
    if (!accel || !curvature)
        return fail(WM_ERR_NULL, "accel/curvature output is NULL");
    CHECK(check_dt(dt));
    if (batch->total_objects > 0)
        wm::launch_inverse(batch->total_objects, *cur, *next, dt, accel, curvature, valid_out, (hipStream_t)stream);
    return device_status("wm_inverse_action");
}

int wm_step_delta(const wm_batch *batch, const wm_state *cur, const wm_delta_action *act, const wm_state *log_next,
                  float dt, wm_state *next, void *stream)
{
    CHECK(check_batch(batch));
    CHECK(check_state(cur, "cur"));
    CHECK(check_state(log_next, "log_next"));
    CHECK(check_state(next, "next"));
    if (!act || !act->dx || !act->dy || !act->dyaw || !act->controlled)
        return fail(WM_ERR_NULL, "delta action is NULL or has a NULL member");
    CHECK(check_dt(dt));
    if (next->x == cur->x)
        return fail(WM_ERR_RANGE, "next must not alias cur");
    wm::launch_delta_step(*batch, *cur, *act, *log_next, *next, dt, (hipStream_t)stream);
    return device_status("wm_step_delta");
}

int wm_inverse_delta(const wm_batch *batch, const wm_state *cur, const wm_state *next, float *dx, float *dy,
                     float *dyaw, uint8_t *valid_out, void *stream)
{
    CHECK(check_batch(batch));
    CHECK(check_state(cur, "cur"));
    CHECK(check_state(next, "next"));
    if (!dx || !dy || !dyaw)
        return fail(WM_ERR_NULL, "dx/dy/dyaw output is NULL");
    if (batch->total_objects > 0)
        wm::launch_delta_inverse(batch->total_objects, *cur, *next, dx, dy, dyaw, valid_out, (hipStream_t)stream);
    return device_status("wm_inverse_delta");
}

int wm_discretize(const float *values, int32_t n, float lo, float hi, int32_t bins, int32_t *index, float *snapped,
                  void *stream)
{
    if (n < 0)
        return fail(WM_ERR_RANGE, "n = %d < 0", n);
    if (n > 0 && (!values || !index))
        return fail(WM_ERR_NULL, "values or index is NULL");
    if (bins < 2)
        return fail(WM_ERR_RANGE, "bins = %d < 2", bins);
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi))
        return fail(WM_ERR_RANGE, "need finite lo < hi (lo = %g, hi = %g)", (double)lo, (double)hi);
    volatile float span = hi - lo;
    volatile float scale = (float)(bins - 1) / span;
    volatile float step = span / (float)(bins - 1);
    if (n > 0)
        wm::launch_discretize(n, values, lo, scale, step, bins, index, snapped, (hipStream_t)stream);
    return device_status("wm_discretize");
}

int wm_overlap(const wm_batch *batch, const wm_state *st, const int64_t *pair_off, float *margin, uint8_t *mask,
               uint8_t *collision, float *max_margin, void *stream)
{
    CHECK(check_batch(batch));
    CHECK(check_state(st, "state"));
    if ((margin || mask) && !pair_off)
        return fail(WM_ERR_NULL, "pair_off is NULL but a margin/mask matrix was requested");
    if (!margin && !mask && !collision && !max_margin)
        return ok();
    wm::OverlapArgs o{batch->obj_off, *st, pair_off, margin, mask, collision, max_margin, batch->max_objects, 64};
    wm::launch_overlap(*batch, o, (hipStream_t)stream);
    return device_status("wm_overlap");
}

int wm_offroad(const wm_batch *batch, const wm_state *st, const wm_roadgraph *rg, uint8_t *offroad, float *margin,
               int32_t *nearest_idx, const wm_tuning *tune, void *ws, size_t ws_bytes, void *stream)
{
    CHECK(check_batch(batch));
    CHECK(check_state(st, "state"));
    if (!rg)
        return fail(WM_ERR_NULL, "roadgraph is NULL");
    CHECK(check_rg(rg));
    Tune tn;
    CHECK(resolve_tune(batch, tune, 1024, &tn));
    const wm::WsLayout L = wm::ws_layout(batch->num_scenarios, batch->total_objects, batch->total_rg_points, 0, 0);
    CHECK(check_ws(ws, ws_bytes, L.total));
    if (!offroad && !margin && !nearest_idx)
        return ok();
    hipStream_t s = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)ws;
    wm::launch_compact_edges(*batch, *rg, w, L, s);
    wm::launch_edge_boxes(*batch, w, L, s);
    wm::OffroadArgs o{batch->obj_off, batch->rg_off, *st, wm::ws_edges(w, L), offroad, margin, nearest_idx, tn.G,
                      tn.CW};
    {
        ProfScope ps(WM_PROF_OFFROAD, s);
        wm::launch_offroad(*batch, o, s);
    }
    return device_status("wm_offroad");
}

static int observe_checks(const wm_batch *batch, const wm_roadgraph *rg, const int32_t *ego, int32_t E, int32_t k,
                          int32_t T, const int32_t *rg_idx)
{
    if (!rg)
        return fail(WM_ERR_NULL, "roadgraph is NULL");
    CHECK(check_rg(rg));
    if (!ego || !rg_idx)
        return fail(WM_ERR_NULL, "ego or rg_idx is NULL");
    if (E < 1 || k < 1 || T < 1)
        return fail(WM_ERR_RANGE, "E = %d, k = %d and T = %d must be >= 1", E, k, T);
    if (T > 65535)
        return fail(WM_ERR_UNSUPPORTED, "T = %d > 65535", T);
    if (k > WM_MAX_TOPK)
        return fail(WM_ERR_UNSUPPORTED, "k = %d > %d", k, WM_MAX_TOPK);
    if (batch->max_rg_points > WM_MAX_OBSERVE_POINTS)
        return fail(WM_ERR_UNSUPPORTED, "max_rg_points = %d > %d", batch->max_rg_points, WM_MAX_OBSERVE_POINTS);
    const long long slots = (long long)batch->num_scenarios * E;
    if (slots * T * (k > 8 ? k : 8) > 0x7fffffffLL || slots * T * batch->max_objects * 8 > 0x7fffffffLL * 4)
        return fail(WM_ERR_UNSUPPORTED, "T * S * E * k too large");
    return WM_OK;
}

int wm_observe_seq(const wm_batch *batch, const wm_state *st, int32_t T, const wm_roadgraph *rg, const int32_t *ego,
                   int32_t E, int32_t k, int32_t *rg_idx, float *rg_feat, float *obj_feat, void *stream)
{
    CHECK(check_batch(batch));
    CHECK(check_state(st, "state"));
    CHECK(observe_checks(batch, rg, ego, E, k, T, rg_idx));
    wm::ObserveArgs a{batch->obj_off, batch->rg_off, *st, *rg, ego, E, k, batch->max_objects, rg_idx, rg_feat,
                      obj_feat, (long)batch->total_objects, (long)batch->num_scenarios};
    {
        ProfScope ps(WM_PROF_OBSERVE, (hipStream_t)stream);
        wm::launch_observe(*batch, a, T, (hipStream_t)stream);
    }
    return device_status("wm_observe");
}

int wm_observe(const wm_batch *batch, const wm_state *st, const wm_roadgraph *rg, const int32_t *ego, int32_t E,
               int32_t k, int32_t *rg_idx, float *rg_feat, float *obj_feat, void *stream)
{
    return wm_observe_seq(batch, st, 1, rg, ego, E, k, rg_idx, rg_feat, obj_feat, stream);
}

int wm_step_observe(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
                    const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *metrics, const int32_t *ego,
                    int32_t E, int32_t k, int32_t *rg_idx, float *rg_feat, float *obj_feat, void *ws,
                    size_t ws_bytes, void *stream)
{
    // every host-visible check of both parts runs before the first launch
    CHECK(check_batch(batch));
    CHECK(observe_checks(batch, rg, ego, E, k, 1, rg_idx));
    CHECK(step_impl(batch, cur, act, log_next, rg, dt, next, metrics, ws, ws_bytes, stream, StepWs::Prepared));
    wm::ObserveArgs a{batch->obj_off, batch->rg_off, *next, *rg, ego, E, k, batch->max_objects, rg_idx, rg_feat,
                      obj_feat, (long)batch->total_objects, (long)batch->num_scenarios};
    {
        ProfScope ps(WM_PROF_OBSERVE, (hipStream_t)stream);
        wm::launch_observe(*batch, a, 1, (hipStream_t)stream);
    }
    return device_status("wm_step_observe");
}

static int rollout_checks(const wm_batch *batch, const wm_state *init, const wm_action *act_seq,
                          const wm_state *log_seq, int32_t T, float dt, int32_t ckpt_every)
{
    CHECK(check_batch(batch));
    CHECK(check_state(init, "init"));
    CHECK(check_state(log_seq, "log_seq"));
    if (!act_seq || !act_seq->accel || !act_seq->curvature || !act_seq->controlled)
        return fail(WM_ERR_NULL, "act_seq is NULL or has a NULL member");
    if (T < 1)
        return fail(WM_ERR_RANGE, "T = %d < 1", T);
    if (ckpt_every < 0)
        return fail(WM_ERR_RANGE, "ckpt_every = %d < 0", ckpt_every);
    if ((long long)(T + 1) * batch->total_objects > 0x7fffffffLL)
        return fail(WM_ERR_UNSUPPORTED, "(T + 1) * total_objects exceeds int32 indexing");
    return check_dt(dt);
}

static int rollout_impl(const wm_batch *batch, const wm_state *init, const wm_action *act_seq,
                        const wm_state *log_seq, const wm_roadgraph *rg, int32_t T, float dt, int32_t ckpt_every,
                        wm_state *ckpt, wm_state *traj, wm_metrics *met_seq, float *loss, const wm_idm *idm,
                        const wm_tuning *tune, void *ws, size_t ws_bytes, void *stream, bool force_off = false)
{
    CHECK(rollout_checks(batch, init, act_seq, log_seq, T, dt, ckpt_every));
    if (rg)
        CHECK(check_rg(rg));
    if (ckpt) {
        CHECK(check_state(ckpt, "ckpt"));
        if (ckpt_every < 1)
            return fail(WM_ERR_RANGE, "ckpt given but ckpt_every = %d < 1", ckpt_every);
    }
    if (traj)
        CHECK(check_state(traj, "traj"));
    Tune tn;
    CHECK(resolve_tune(batch, tune, 512, &tn));
    const wm::WsLayout L =
        wm::ws_layout(batch->num_scenarios, batch->total_objects, batch->total_rg_points, T, ckpt_every);
    CHECK(check_ws(ws, ws_bytes, L.total));
    const size_t lds = wm::rollout_lds_bytes(batch->max_objects, tn.G, tn.CW);
    if (lds > 160 * 1024)
        return fail(WM_ERR_UNSUPPORTED, "rollout needs %zu bytes of LDS", lds);
    hipStream_t s = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)ws;
    // the off-road scan runs only when an output needs it
    // (force_off: the autotuner times the scan without outputs)
    const bool want_off =
        rg && (force_off || (met_seq && (met_seq->offroad || met_seq->offroad_margin || met_seq->reward)));
    if (want_off) {
        wm::launch_compact_edges(*batch, *rg, w, L, s);
        wm::launch_edge_boxes(*batch, w, L, s);
    }
    wm::launch_build_units(*batch, 64 * tn.CW, want_off ? (const int32_t *)(w + L.ecount) : nullptr, w, L, s);
    wm::RollArgs a{};
    a.S = batch->num_scenarios;
    a.n = batch->total_objects;
    a.T = T;
    a.ckpt_every = ckpt_every;
    a.maxN = batch->max_objects;
    a.G = tn.G;
    a.CW = tn.CW;
    a.dt = dt;
    a.obj_off = batch->obj_off;
    a.rg_off = batch->rg_off;
    a.init = *init;
    a.act = *act_seq;
    a.log = *log_seq;
    a.has_rg = want_off;
    a.has_ckpt = ckpt != nullptr;
    a.has_traj = traj != nullptr;
    a.want_loss = loss != nullptr;
    a.E = wm::ws_edges(w, L);
    if (ckpt)
        a.ckpt = *ckpt;
    if (traj)
        a.traj = *traj;
    if (met_seq)
        a.met = *met_seq;
    a.lossp = (float *)(w + L.lossp);
    a.uoff = (const int32_t *)(w + L.uoff);
    a.units = (const int2 *)(w + L.units);
    a.counter = (int32_t *)(w + L.counter);
    if (idm) {
        a.has_idm = 1;
        a.idm = *idm;
        a.idmP = (const float4 *)(w + L.idmP);
        a.idmA = (const uint8_t *)(w + L.idmA);
        wm::launch_idm_paths(batch->total_objects, T, *log_seq, act_seq->controlled, (float4 *)(w + L.idmP),
                             (uint8_t *)(w + L.idmA), s);
    }
    const int U = 64 * tn.CW;
    const int bound = batch->total_objects / U + batch->num_scenarios;
    const int grid = wm::rollout_grid(tn.G, tn.CW, batch->max_objects, bound);
    {
        ProfScope ps(WM_PROF_ROLLOUT, s);
        wm::launch_rollout(a, grid, s);
    }
    if (loss)
        wm::launch_loss_reduce(batch->num_scenarios, a.uoff, a.lossp, loss, s);
    return device_status(idm ? "wm_rollout_idm" : "wm_rollout");
}

int wm_rollout(const wm_batch *batch, const wm_state *init, const wm_action *act_seq, const wm_state *log_seq,
               const wm_roadgraph *rg, int32_t T, float dt, int32_t ckpt_every, wm_state *ckpt, wm_state *traj,
               wm_metrics *met_seq, float *loss, const wm_tuning *tune, void *ws, size_t ws_bytes, void *stream)
{
    return rollout_impl(batch, init, act_seq, log_seq, rg, T, dt, ckpt_every, ckpt, traj, met_seq, loss, nullptr,
                        tune, ws, ws_bytes, stream);
}

int wm_rollout_scan_counts(const wm_batch *batch, const void *ws, size_t ws_bytes, uint64_t *counts, void *stream)
{
    CHECK(check_batch(batch));
    if (!ws || !counts)
        return fail(WM_ERR_NULL, "wm_rollout_scan_counts: ws or counts is NULL");
    // the queue counters sit before every section that depends on T or the
    // checkpoint interval
    const wm::WsLayout L = wm::ws_layout(batch->num_scenarios, batch->total_objects, batch->total_rg_points, 0, 0);
    const size_t at = L.counter + sizeof(int32_t) * wm::kRollCounts;
    if (ws_bytes < at + sizeof(uint64_t) * wm::kRollCountN)
        return fail(WM_ERR_WORKSPACE, "wm_rollout_scan_counts: workspace of %zu bytes is too small", ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(counts, (const unsigned char *)ws + at, sizeof(uint64_t) * wm::kRollCountN,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return fail(WM_ERR_DEVICE, "wm_rollout_scan_counts: %s", hipGetErrorString(e));
    return ok();
}

int wm_rollout_idm(const wm_batch *batch, const wm_state *init, const wm_action *act_seq, const wm_state *log_seq,
                   const wm_roadgraph *rg, int32_t T, float dt, const wm_idm *idm, wm_state *traj,
                   wm_metrics *met_seq, const wm_tuning *tune, void *ws, size_t ws_bytes, void *stream)
{
    if (!idm)
        return fail(WM_ERR_NULL, "idm parameters are NULL");
    const float pos[] = {idm->desired_speed, idm->max_accel, idm->comfort_decel, idm->exponent, idm->max_brake,
                         idm->lookahead_step};
    for (float v : pos)
        if (!(v > 0.f) || !std::isfinite(v))
            return fail(WM_ERR_RANGE, "idm: speeds, accelerations, exponent and step must be finite and > 0");
    if (!(idm->min_gap >= 0.f) || !(idm->time_headway >= 0.f) || !std::isfinite(idm->min_gap) ||
        !std::isfinite(idm->time_headway))
        return fail(WM_ERR_RANGE, "idm: min_gap and time_headway must be finite and >= 0");
    if (idm->lookahead_poses < 1 || idm->lookahead_poses > WM_MAX_IDM_POSES)
        return fail(WM_ERR_RANGE, "idm: lookahead_poses = %d not in [1, %d]", idm->lookahead_poses,
                    WM_MAX_IDM_POSES);
    return rollout_impl(batch, init, act_seq, log_seq, rg, T, dt, 0, nullptr, traj, met_seq, nullptr, idm, tune, ws,
                        ws_bytes, stream);
}

int wm_rollout_backward(const wm_batch *batch, const wm_state *init, const wm_action *act_seq,
                        const wm_state *log_seq, int32_t T, float dt, int32_t ckpt_every, const wm_state *ckpt,
                        const float *dloss, float *grad_accel, float *grad_curvature, void *ws, size_t ws_bytes,
                        void *stream)
{
    CHECK(rollout_checks(batch, init, act_seq, log_seq, T, dt, ckpt_every));
    CHECK(check_state(ckpt, "ckpt"));
    if (ckpt_every < 1)
        return fail(WM_ERR_RANGE, "ckpt_every = %d < 1", ckpt_every);
    if (!dloss || !grad_accel || !grad_curvature)
        return fail(WM_ERR_NULL, "dloss or a gradient output is NULL");
    const wm::WsLayout L =
        wm::ws_layout(batch->num_scenarios, batch->total_objects, batch->total_rg_points, T, ckpt_every);
    CHECK(check_ws(ws, ws_bytes, L.total));
    wm::BackwardArgs a{};
    a.S = batch->num_scenarios;
    a.n = batch->total_objects;
    a.T = T;
    a.K = ckpt_every;
    a.maxN = batch->max_objects;
    a.SB = wm::backward_block_steps(a.maxN, a.K);
    a.dt = dt;
    a.obj_off = batch->obj_off;
    a.init = *init;
    a.act = *act_seq;
    a.log = *log_seq;
    a.ckpt = *ckpt;
    a.dloss = dloss;
    a.grad_a = grad_accel;
    a.grad_k = grad_curvature;
    a.rec = (float *)((unsigned char *)ws + L.seg);
    a.part = a.rec + (size_t)wm::kRecFields * T * batch->total_objects;
    {
        ProfScope ps(WM_PROF_BACKWARD, (hipStream_t)stream);
        wm::launch_backward(a, (hipStream_t)stream);
    }
    return device_status("wm_rollout_backward");
}

int wm_autotune(const wm_batch *batch, const wm_state *init, const wm_action *act_seq, const wm_state *log_seq,
                const wm_roadgraph *rg, int32_t T, float dt, void *ws, size_t ws_bytes, wm_tuning *best,
                void *stream)
{
    CHECK(rollout_checks(batch, init, act_seq, log_seq, T, dt, 0));
    const wm::WsLayout L = wm::ws_layout(batch->num_scenarios, batch->total_objects, batch->total_rg_points, T, 0);
    CHECK(check_ws(ws, ws_bytes, L.total));
    {
        // a tuning kept by an earlier process (WM_TUNE_CACHE) is taken as is
        std::lock_guard<std::mutex> lk(g_tune_mu);
        Tune cached;
        if (tune_cache_lookup(tune_key(batch), &cached)) {
            g_tune_table[tune_key(batch)] = cached;
            if (best)
                *best = wm_tuning{64 * cached.CW, cached.G};
            return ok();
        }
    }
    static const int cand[][2] = {{64, 2}, {64, 4}, {64, 8}, {128, 1}, {128, 2}, {128, 4}, {256, 1}, {256, 2}};
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return device_status("wm_autotune: event");
    float best_ms = 1e30f;
    wm_tuning pick{64, 8};
    for (const auto &c : cand) {
        wm_tuning t{c[0], c[1]};
        if (wm::rollout_lds_bytes(batch->max_objects, t.edge_splits, t.unit_objects / 64) > 160 * 1024)
            continue;
        int rc = rollout_impl(batch, init, act_seq, log_seq, rg, T, dt, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                              &t, ws, ws_bytes, stream, true);
        if (rc != WM_OK)
            break;
        hipEventRecord(e0, s);
        for (int r = 0; r < 2; ++r)
            (void)rollout_impl(batch, init, act_seq, log_seq, rg, T, dt, 0, nullptr, nullptr, nullptr, nullptr,
                               nullptr, &t, ws, ws_bytes, stream, true);
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            pick = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    const int rc = device_status("wm_autotune");
    if (rc != WM_OK)
        return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_table[tune_key(batch)] = Tune{pick.edge_splits, pick.unit_objects / 64};
        tune_cache_store(tune_key(batch), pick);
    }
    if (best)
        *best = pick;
    return ok();
}

} // extern "C"
