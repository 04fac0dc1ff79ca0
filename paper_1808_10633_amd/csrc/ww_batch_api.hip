// ww_batch_api.hip -- C ABI of the batched form: arena layout, the
// largest-first patch order the resident blocks take their work from, graph
// capture and replay of whole RK4 steps, and the autotuner of the launch
// shape.
#include "../../include/wombat_weno.h"
#include "ww_batch.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

using ww::BatchArgs;
using ww::FaceBox;
using ww::Geom;
using ww::PatchDesc;

struct wombat_weno_batch {
    wombat_weno_config cfg;
    int npatch;
    std::vector<int> dims;          // 3 per patch
    std::vector<long> soff;         // arena offset of each patch
    std::vector<PatchDesc> hpd;
    long arena;                     // elements per arena
    size_t esize;
    long slot_elems;
    int ncu;
    int ft, bpc, nblocks;           // launch shape: faces per y/z tile, blocks per CU
    int maxblocks;
    PatchDesc *pd;
    int *order;            // patches by decreasing cost
    int32_t *counters;     // work counters of the 4 stages of a step
    void *work[3];                  // A, B, acc arenas
    void *scratch;
    double *dt;
    int32_t *flag;
    hipStream_t st, cap;            // user stream, capture stream
    hipGraph_t graph;
    hipGraphExec_t exec;
    void *graph_arena;
    hipEvent_t ev[2];
    int sticky;
    std::string err;
};

namespace {

thread_local std::string g_berr;

int bfail(wombat_weno_batch_t *b, int code, const std::string &m)
{
    if (b) b->err = m; else g_berr = m;
    return code;
}

int bhip(wombat_weno_batch_t *b, hipError_t e, const char *what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    if (b) { b->sticky = 1; b->err = buf; } else g_berr = buf;
    return WW_ERR_HIP;
}

#define WB_CHECK(b, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return bhip(b, e_, #call);    \
    } while (0)

struct DevGuard {
    int prev = -1;
    bool ok = true;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DevGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void patch_geom(const int n[3], double dl, Geom &G, FaceBox F[3])
{
    int N[3];
    for (int d = 0; d < 3; ++d) {
        G.n[d] = n[d];
        G.act[d] = 1;
        G.g[d] = 3;
        G.dl[d] = dl;
        G.idl[d] = 1.0 / dl;
        N[d] = n[d] + 6;
    }
    G.s[0] = 1;
    G.s[1] = N[0];
    G.s[2] = (long)N[0] * N[1];
    G.sv = (long)N[0] * N[1] * N[2];
    G.base = 3 + 3 * G.s[1] + 3 * G.s[2];
    for (int d = 0; d < 3; ++d) {
        FaceBox &B = F[d];
        for (int e = 0; e < 3; ++e) {
            if (e == d) { B.lo[e] = 0; B.cnt[e] = n[e] + 1; }
            else { B.lo[e] = -1; B.cnt[e] = n[e] + 2; }
        }
        B.s[0] = 1;
        B.s[1] = B.cnt[0];
        B.s[2] = (long)B.cnt[0] * B.cnt[1];
        B.sc = (long)B.cnt[0] * B.cnt[1] * B.cnt[2];
    }
}

double patch_cost(const int n[3])
{
    double c = 0.0;
    for (int d = 0; d < 3; ++d) {
        double f = n[d] + 1.0;
        for (int e = 0; e < 3; ++e) if (e != d) f *= n[e] + 2.0;
        c += f;
    }
    return c;
}

// Patches by decreasing estimated cost (ties by index).
void make_order(const std::vector<int> &dims, std::vector<int> &order)
{
    const int np = (int)dims.size() / 3;
    order.resize(np);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> cost(np);
    for (int p = 0; p < np; ++p) cost[p] = patch_cost(&dims[3 * p]);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
}

int set_shape(wombat_weno_batch_t *b, int ft, int bpc)
{
    int occ = 0;
    hipError_t e = b->cfg.precision == WW_FP64 ? ww::batch_occupancy<double>(ft, &occ)
                                               : ww::batch_occupancy<float>(ft, &occ);
    if (e != hipSuccess) return bhip(b, e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (occ < 1) return bfail(b, WW_ERR_UNSUPPORTED, "batched kernel does not fit on a CU");
    if (bpc > occ) bpc = occ;
    WB_CHECK(b, hipStreamSynchronize(b->st));      // no launch may still run with the old shape
    int nblocks = bpc * b->ncu;
    if (nblocks > b->maxblocks) nblocks = b->maxblocks;
    b->ft = ft;
    b->bpc = bpc;
    b->nblocks = nblocks;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->graph_arena = nullptr;
    return WW_OK;
}

template <typename T>
BatchArgs<T> stage_args(wombat_weno_batch_t *b, int s, T *u0, T *us, T *acc, T *out, double bw, double cw)
{
    BatchArgs<T> a;
    a.pd = b->pd;
    a.order = b->order;
    a.npatch = (int)(b->dims.size() / 3);
    a.counter = b->counters + s;
    a.u0 = u0;
    a.us = us;
    a.acc = acc;
    a.out = out;
    a.scratch = (T *)b->scratch;
    a.slot_elems = b->slot_elems;
    a.dt = b->dt;
    a.flag = b->flag;
    a.cfl = b->cfg.cfl;
    a.s = s;
    a.bw = bw;
    a.cw = cw;
    a.P = ww::Phys{ b->cfg.gamma, b->cfg.eps, 1.0 / (b->cfg.gamma - 1.0) };
    return a;
}

template <typename T>
int launch_step_t(wombat_weno_batch_t *b, T *u, hipStream_t st)
{
    static const double bw[4] = { 1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 0.0 };
    static const double cw[4] = { 0.5, 0.5, 1.0, 1.0 / 6.0 };
    T *A = (T *)b->work[0], *B = (T *)b->work[1], *acc = (T *)b->work[2];
    T *in[4] = { u, A, B, A };
    T *out[4] = { A, B, A, u };
    WB_CHECK(b, ww::launch_batch_reset(b->counters, 4, st));
    for (int s = 0; s < 4; ++s)
        WB_CHECK(b, ww::launch_batch_stage<T>(stage_args<T>(b, s, u, in[s], acc, out[s], bw[s], cw[s]), b->ft,
                                              b->nblocks, st));
    return WW_OK;
}

// Autotuner set-up: A = a copy of u, then stage 0 of a step from A (which
// computes every patch's dt and leaves U_2 in B).
template <typename T>
int tune_prepare_t(wombat_weno_batch_t *b, const T *u)
{
    T *A = (T *)b->work[0], *B = (T *)b->work[1], *acc = (T *)b->work[2];
    WB_CHECK(b, hipMemcpyAsync(A, u, b->esize * b->arena, hipMemcpyDeviceToDevice, b->st));
    WB_CHECK(b, ww::launch_batch_reset(b->counters, 4, b->st));
    WB_CHECK(b, ww::launch_batch_stage<T>(stage_args<T>(b, 0, A, A, acc, B, 1.0 / 6.0, 0.5), b->ft, b->nblocks,
                                          b->st));
    return WW_OK;
}

// One timed launch of the second stage's form on (u0 = A, us = B, acc), with
// zero RK weights: acc and out = A keep their values, so every launch does
// the same work.
template <typename T>
int tune_stage_t(wombat_weno_batch_t *b, float *ms)
{
    T *A = (T *)b->work[0], *B = (T *)b->work[1], *acc = (T *)b->work[2];
    WB_CHECK(b, ww::launch_batch_reset(b->counters + 1, 1, b->st));
    WB_CHECK(b, hipEventRecord(b->ev[0], b->st));
    WB_CHECK(b, ww::launch_batch_stage<T>(stage_args<T>(b, 1, A, B, acc, A, 0.0, 0.0), b->ft, b->nblocks, b->st));
    WB_CHECK(b, hipEventRecord(b->ev[1], b->st));
    WB_CHECK(b, hipEventSynchronize(b->ev[1]));
    WB_CHECK(b, hipEventElapsedTime(ms, b->ev[0], b->ev[1]));
    return WW_OK;
}

int launch_step(wombat_weno_batch_t *b, void *u, hipStream_t st)
{
    return b->cfg.precision == WW_FP64 ? launch_step_t<double>(b, (double *)u, st)
                                       : launch_step_t<float>(b, (float *)u, st);
}

int precheck(wombat_weno_batch_t *b)
{
    if (!b) return bfail(nullptr, WW_ERR_INVALID_ARG, "batch is NULL");
    if (b->sticky) return WW_ERR_HIP;
    return WW_OK;
}

void release(wombat_weno_batch_t *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (int i = 0; i < 3; ++i) if (b->work[i]) (void)hipFree(b->work[i]);
    if (b->scratch) (void)hipFree(b->scratch);
    if (b->pd) (void)hipFree(b->pd);
    if (b->order) (void)hipFree(b->order);
    if (b->counters) (void)hipFree(b->counters);
    if (b->dt) (void)hipFree(b->dt);
    if (b->flag) (void)hipFree(b->flag);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int i = 0; i < 2; ++i) if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
}

std::string tune_key(const wombat_weno_batch_t *b)
{
    unsigned long long h = 1469598103934665603ULL;
    for (int v : b->dims) { h ^= (unsigned)v; h *= 1099511628211ULL; }
    char buf[160];
    snprintf(buf, sizeof buf, "gfx950|%s|%d|%016llx", b->cfg.precision == WW_FP64 ? "fp64" : "fp32",
             b->npatch, h);
    return buf;
}

// Tiny JSON cache: one line per entry, {"key": "...", "ft": F, "bpc": B, "ms": M}.
bool cache_lookup(const char *path, const std::string &key, int &ft, int &bpc)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, ("\"" + key + "\"").c_str())) continue;
        const char *a = strstr(line, "\"ft\":"), *c = strstr(line, "\"bpc\":");
        if (a && c) { ft = atoi(a + 5); bpc = atoi(c + 6); found = true; }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, int ft, int bpc, double ms)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"ft\": %d, \"bpc\": %d, \"ms\": %.4f}\n", key.c_str(), ft, bpc, ms);
    fclose(f);
}

}  // namespace

extern "C" {

int wombat_weno_batch_init(const wombat_weno_config *cfg, int npatch, const int32_t *dims,
                           wombat_weno_batch_t **out)
{
    if (!cfg || !dims || !out) return bfail(nullptr, WW_ERR_INVALID_ARG, "NULL argument");
    if (npatch < 1 || npatch > (1 << 22)) return bfail(nullptr, WW_ERR_INVALID_ARG, "npatch must be in 1..4194304");
    if (!(cfg->dx > 0.0) || !std::isfinite(cfg->dx)) return bfail(nullptr, WW_ERR_INVALID_ARG, "dx must be finite and > 0");
    if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0) || !(cfg->cfl <= 1.0) || !(cfg->eps > 0.0))
        return bfail(nullptr, WW_ERR_INVALID_ARG, "need gamma > 1, cfl in (0,1], eps > 0");
    if (cfg->precision != WW_FP64 && cfg->precision != WW_FP32_MIXED)
        return bfail(nullptr, WW_ERR_INVALID_ARG, "unknown precision");
    if (cfg->weights != WW_WEIGHTS_JS)
        return bfail(nullptr, WW_ERR_UNSUPPORTED, "the batched form uses the WENO-JS weights only");
    if (cfg->integrator != WW_RK4)
        return bfail(nullptr, WW_ERR_UNSUPPORTED, "the batched form uses the RK4 step only");
    if (cfg->lf_speed != WW_LF_LOCAL)
        return bfail(nullptr, WW_ERR_UNSUPPORTED, "the batched form uses the per-stencil LF speeds only");
    if (cfg->b_storage != WW_B_CELL)
        return bfail(nullptr, WW_ERR_UNSUPPORTED, "the batched form stores cell-centred B only");
    for (int p = 0; p < npatch; ++p)
        for (int d = 0; d < 3; ++d)
            if (dims[3 * p + d] < 4 || dims[3 * p + d] > 1024)
                return bfail(nullptr, WW_ERR_INVALID_ARG, "patch edges must be in 4..1024 cells");
    wombat_weno_batch_t *b = new (std::nothrow) wombat_weno_batch();
    if (!b) return bfail(nullptr, WW_ERR_OOM, "host allocation failed");
    b->cfg = *cfg;
    b->npatch = npatch;
    b->dims.assign(dims, dims + 3 * npatch);
    b->esize = cfg->precision == WW_FP64 ? 8 : 4;
    b->st = (hipStream_t)cfg->stream;
    DevGuard dg(cfg->device);
    if (!dg.ok) { delete b; return bfail(nullptr, WW_ERR_HIP, "hipSetDevice failed"); }
    // arena layout (each patch aligned to 64 elements) and patch table
    long off = 0, slot = 0;
    b->hpd.resize(npatch);
    b->soff.resize(npatch);
    for (int p = 0; p < npatch; ++p) {
        const int *n = &b->dims[3 * p];
        PatchDesc &D = b->hpd[p];
        memset(&D, 0, sizeof D);
        patch_geom(n, cfg->dx, D.G, D.F);
        D.soff = off;
        D.xflat = ww::batch_xflat_ok(n[0], (long)D.F[0].cnt[1] * D.F[0].cnt[2]) ? 1 : 0;
        b->soff[p] = off;
        off += (8 * D.G.sv + 63) / 64 * 64;
        slot = std::max(slot, (long)ww::NFC * (D.F[0].sc + D.F[1].sc + D.F[2].sc));
    }
    b->arena = off;
    b->slot_elems = (slot + 63) / 64 * 64;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess || ncu < 1)
        ncu = 256;
    b->ncu = ncu;
    b->maxblocks = 4 * ncu;
    auto fail_oom = [&](const char *what) {
        release(b);
        delete b;
        return bfail(nullptr, WW_ERR_OOM, std::string("device allocation failed: ") + what);
    };
    ww::alloc_hook_reset();
    for (int i = 0; i < 3; ++i)
        if (ww::dev_alloc(&b->work[i], b->esize * b->arena) != hipSuccess) return fail_oom("work arenas");
    if (ww::dev_alloc(&b->scratch, b->esize * b->slot_elems * b->maxblocks) != hipSuccess) return fail_oom("face scratch");
    if (ww::dev_alloc((void **)&b->pd, sizeof(PatchDesc) * npatch) != hipSuccess) return fail_oom("patch table");
    if (ww::dev_alloc((void **)&b->order, sizeof(int) * npatch) != hipSuccess) return fail_oom("patch order");
    if (ww::dev_alloc((void **)&b->counters, sizeof(int32_t) * 4) != hipSuccess) return fail_oom("work counters");
    if (ww::dev_alloc((void **)&b->dt, sizeof(double) * npatch) != hipSuccess) return fail_oom("dt");
    if (ww::dev_alloc((void **)&b->flag, sizeof(int32_t) * npatch) != hipSuccess) return fail_oom("flags");
    std::vector<int> order;
    make_order(b->dims, order);
    if (hipMemcpy(b->pd, b->hpd.data(), sizeof(PatchDesc) * npatch, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->order, order.data(), sizeof(int) * npatch, hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->ev[0]) != hipSuccess || hipEventCreate(&b->ev[1]) != hipSuccess) {
        release(b);
        delete b;
        return bfail(nullptr, WW_ERR_HIP, "batch set-up failed");
    }
    int rc = set_shape(b, 4, 2);
    if (rc) {
        std::string m = b->err;
        release(b);
        delete b;
        return bfail(nullptr, rc, m);
    }
    *out = b;
    return WW_OK;
}

void wombat_weno_batch_destroy(wombat_weno_batch_t *b)
{
    if (!b) return;
    DevGuard dg(b->cfg.device);
    if (!b->sticky) (void)hipStreamSynchronize(b->st);
    release(b);
    delete b;
}

const char *wombat_weno_batch_last_error(const wombat_weno_batch_t *b)
{
    return b ? b->err.c_str() : g_berr.c_str();
}

int64_t wombat_weno_batch_arena_elems(const wombat_weno_batch_t *b) { return b ? b->arena : -1; }

int64_t wombat_weno_batch_patch_offset(const wombat_weno_batch_t *b, int p)
{
    if (!b || p < 0 || p >= b->npatch) return -1;
    return b->soff[p];
}

int wombat_weno_batch_step(wombat_weno_batch_t *b, void *d_arena)
{
    int rc = precheck(b);
    if (rc) return rc;
    if (!d_arena) return bfail(b, WW_ERR_INVALID_ARG, "d_arena is NULL");
    DevGuard dg(b->cfg.device);
    return launch_step(b, d_arena, b->st);
}

int wombat_weno_batch_graph_steps(wombat_weno_batch_t *b, void *d_arena, int nsteps)
{
    int rc = precheck(b);
    if (rc) return rc;
    if (!d_arena || nsteps < 0) return bfail(b, WW_ERR_INVALID_ARG, "need d_arena and nsteps >= 0");
    DevGuard dg(b->cfg.device);
    if (!b->exec || b->graph_arena != d_arena) {
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        WB_CHECK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        rc = launch_step(b, d_arena, b->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
        b->graph = g;
        WB_CHECK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_arena = d_arena;
    }
    for (int i = 0; i < nsteps; ++i) WB_CHECK(b, hipGraphLaunch(b->exec, b->st));
    return WW_OK;
}

int wombat_weno_batch_dt(wombat_weno_batch_t *b, double *h_dt, int32_t *h_flag)
{
    int rc = precheck(b);
    if (rc) return rc;
    DevGuard dg(b->cfg.device);
    WB_CHECK(b, hipStreamSynchronize(b->st));
    if (h_dt) WB_CHECK(b, hipMemcpy(h_dt, b->dt, sizeof(double) * b->npatch, hipMemcpyDeviceToHost));
    if (h_flag) WB_CHECK(b, hipMemcpy(h_flag, b->flag, sizeof(int32_t) * b->npatch, hipMemcpyDeviceToHost));
    return WW_OK;
}

int wombat_weno_batch_shape(const wombat_weno_batch_t *b, int *ft, int *blocks_per_cu, int *nblocks)
{
    if (!b) return bfail(nullptr, WW_ERR_INVALID_ARG, "batch is NULL");
    if (ft) *ft = b->ft;
    if (blocks_per_cu) *blocks_per_cu = b->bpc;
    if (nblocks) *nblocks = b->nblocks;
    return WW_OK;
}

int wombat_weno_batch_autotune(wombat_weno_batch_t *b, const void *d_arena, const char *cache_path,
                               double *best_ms)
{
    int rc = precheck(b);
    if (rc) return rc;
    if (!d_arena) return bfail(b, WW_ERR_INVALID_ARG, "d_arena is NULL");
    DevGuard dg(b->cfg.device);
    const std::string key = tune_key(b);
    int ft = 0, bpc = 0;
    if (cache_lookup(cache_path, key, ft, bpc) && (ft == 4 || ft == 8 || ft == 12 || ft == 16) && bpc >= 1 &&
        bpc <= 4) {
        if (best_ms) *best_ms = -1.0;
        return set_shape(b, ft, bpc);
    }
    // Every shape is timed on the same work: a copy of the state in the work
    // arenas, advanced through stage 0 once; then per shape one untimed and
    // five timed launches of stage 1 with zero RK weights, ranked by the
    // median.  No allocation.
    const bool f64 = b->cfg.precision == WW_FP64;
    rc = f64 ? tune_prepare_t<double>(b, (const double *)d_arena) : tune_prepare_t<float>(b, (const float *)d_arena);
    if (rc) return rc;
    double best = 1e300;
    int bft = 4, bb = 1;
    const int fts[4] = { 4, 8, 12, 16 };
    constexpr int NT = 5;
    for (int fi = 0; fi < 4; ++fi)
        for (int c = 1; c <= 4; ++c) {
            rc = set_shape(b, fts[fi], c);
            if (rc) return rc;
            if (b->bpc != c) continue;          // beyond the occupancy limit
            float t[NT + 1];
            for (int r = 0; r <= NT; ++r) {
                rc = f64 ? tune_stage_t<double>(b, &t[r]) : tune_stage_t<float>(b, &t[r]);
                if (rc) return rc;
            }
            std::sort(t + 1, t + NT + 1);
            const double med = t[1 + NT / 2];
            if (med < best) { best = med; bft = fts[fi]; bb = c; }
        }
    rc = set_shape(b, bft, bb);
    if (rc) return rc;
    cache_store(cache_path, key, bft, bb, best);
    if (best_ms) *best_ms = best;
    return WW_OK;
}

}  // extern "C"
