// ww_api.hip -- the C ABI of include/wombat_weno.h: validation, context,
// device memory, call order and error reporting.  All device work is
// enqueued on the context's stream; no allocation happens after init.
#include "../../include/wombat_weno.h"
#include "ww_internal.h"
#include "ww_router.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <new>
#include <string>

using ww::FaceBox;
using ww::Geom;
using ww::dev_alloc;

namespace ww {

namespace {
std::atomic<long long> g_allocs{ 0 };   // allocations since the library was loaded
std::atomic<int> g_since_init{ 0 };     // allocations since the latest (batch) init
}  // namespace

static bool alloc_should_fail()
{
    const int k = ++g_since_init;
    const char *f = getenv("WOMBAT_WENO_FAIL_ALLOC");
    return f && atoi(f) == k;
}

hipError_t dev_alloc(void **p, size_t bytes)
{
    ++g_allocs;
    if (alloc_should_fail()) { *p = nullptr; return hipErrorOutOfMemory; }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) *p = nullptr;
    return e;
}

hipError_t host_alloc(void **p, size_t bytes)
{
    ++g_allocs;
    if (alloc_should_fail()) { *p = nullptr; return hipErrorOutOfMemory; }
    hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) *p = nullptr;
    return e;
}

void alloc_hook_reset() { g_since_init = 0; }
long long alloc_total() { return g_allocs.load(); }

}  // namespace ww

struct wombat_weno {
    wombat_weno_config cfg;
    Geom G;
    FaceBox F[3];
    size_t esize;          // bytes per state element
    long elems;            // elements per state array
    void *work[3];         // state-sized work arrays
    void *ff[3];           // face fluxes per direction
    double *part;          // reduction partials (nblk x 8)
    int32_t *partflag;     // reduction flags (nblk)
    double *dsmall;        // [0] dt, [1..8] sums / divb, flag at dflag
    int32_t *dflag;
    double *hsmall;        // pinned host mirror of dsmall (16 doubles + flag)
    int nblk;
    hipEvent_t ev[2];      // kernel timing
    int router;            // learned routing switched on
    char *router_pk;       // its parameters, packed in MFMA operand order
    float router_thr;      // logit threshold of "troubled"
    int router_force;      // 0 routed, +1 all full WENO, -1 all linear (same kernel)
    int32_t *nsmooth;      // per-block smooth counts of the last learned sweeps
    long nsm_blocks[3];
    void *backup;          // u at the start of a routed step (allocated with the router)
    unsigned long long *queue;   // troubled interfaces of the current routed sweep
    int32_t *qcount;       // its length
    unsigned char *rmask;  // routing decisions per face, the three directions one after another
    int router_reuse;      // stages 2-4 of a step: reuse the decisions of its first stage
    int64_t fallbacks;     // routed steps redone with full WENO
    double *lfg;           // global LF speeds: partials, then 7 per direction (WW_LF_GLOBAL only)
    int slab;              // z-slab mode: planes per slab (0: whole box)
    int fuse;              // the x sweep does the rho, m, E update (3-D, long rows, no slabs, no router)
    void *delay;           // slab mode: the last 3 output planes of a slab (8 vars x 3 planes)
    void *cellst;          // WW_B_FACE: the cell-centred state the sweeps read
    hipStream_t st;
    int sticky;            // a HIP error happened: every later call fails
    std::string err;
};

namespace {

thread_local std::string g_err;

int fail_ctx(wombat_weno_t *c, int code, const std::string &msg)
{
    if (c) c->err = msg; else g_err = msg;
    return code;
}

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

int hip_fail(wombat_weno_t *c, hipError_t e, const char *what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    if (c) { c->sticky = 1; c->err = buf; } else g_err = buf;
    return WW_ERR_HIP;
}

#define WW_CHECK(ctx, call)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

int validate(const wombat_weno_config *c, std::string &why) { return ww::validate_config(c, why); }

}  // namespace

void ww::set_global_error(const std::string &msg) { g_err = msg; }

int ww::validate_config(const wombat_weno_config *c, std::string &why)
{
    if (!c) { why = "config is NULL"; return WW_ERR_INVALID_ARG; }
    const int n[3] = { c->nx, c->ny, c->nz };
    const double dl[3] = { c->dx, c->dy, c->dz };
    int nact = 0;
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1) { why = "cell counts must be >= 1"; return WW_ERR_INVALID_ARG; }
        if (n[d] == 2) { why = "an active axis needs at least 3 cells"; return WW_ERR_INVALID_ARG; }
        if (n[d] > (1 << 20)) { why = "cell count too large"; return WW_ERR_INVALID_ARG; }
        if (!(dl[d] > 0.0) || !std::isfinite(dl[d])) { why = "cell widths must be finite and > 0"; return WW_ERR_INVALID_ARG; }
        nact += n[d] > 1;
    }
    if (nact == 0) { why = "at least one axis must have more than one cell"; return WW_ERR_INVALID_ARG; }
    if (c->ng != 3) { why = "ng must be 3"; return WW_ERR_INVALID_ARG; }
    if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) { why = "gamma must be > 1"; return WW_ERR_INVALID_ARG; }
    if (!(c->cfl > 0.0) || !(c->cfl <= 1.0)) { why = "cfl must be in (0, 1]"; return WW_ERR_INVALID_ARG; }
    if (!(c->eps > 0.0) || !std::isfinite(c->eps)) { why = "eps must be finite and > 0"; return WW_ERR_INVALID_ARG; }
    if (c->precision != WW_FP64 && c->precision != WW_FP32_MIXED) { why = "unknown precision"; return WW_ERR_INVALID_ARG; }
    if (c->weights != WW_WEIGHTS_JS && c->weights != WW_WEIGHTS_Z) { why = "unknown weights"; return WW_ERR_INVALID_ARG; }
    if (c->integrator != WW_RK4 && c->integrator != WW_SSPRK3) { why = "unknown integrator"; return WW_ERR_INVALID_ARG; }
    if (c->lf_speed != WW_LF_LOCAL && c->lf_speed != WW_LF_GLOBAL) { why = "unknown lf_speed"; return WW_ERR_INVALID_ARG; }
    if (c->learned != 0 && c->learned != 1) { why = "learned must be 0 or 1"; return WW_ERR_INVALID_ARG; }
    if (c->slab_planes < 0 || (c->slab_planes > 0 && c->slab_planes < 3)) {
        why = "slab_planes must be 0 or >= 3";
        return WW_ERR_INVALID_ARG;
    }
    if (c->slab_planes > 0 && c->nz < 3) { why = "slab_planes needs an active z axis"; return WW_ERR_INVALID_ARG; }
    if (c->b_storage != WW_B_CELL && c->b_storage != WW_B_FACE) { why = "unknown b_storage"; return WW_ERR_INVALID_ARG; }
    bool user = false;
    for (int f = 0; f < 6; ++f) {
        if (c->bc[f] < 0 || c->bc[f] > 2) { why = "unknown boundary condition"; return WW_ERR_INVALID_ARG; }
        user = user || c->bc[f] == WW_BC_USER;
    }
    for (int d = 0; d < 3; ++d)
        if ((c->bc[2 * d] == WW_BC_PERIODIC) != (c->bc[2 * d + 1] == WW_BC_PERIODIC)) {
            why = "periodic boundaries must be set on both faces of an axis";
            return WW_ERR_INVALID_ARG;
        }
    if (user && !c->user_bc) { why = "a WW_BC_USER face needs user_bc"; return WW_ERR_INVALID_ARG; }
    if (c->device < 0) { why = "device must be >= 0"; return WW_ERR_INVALID_ARG; }
    return WW_OK;
}

namespace {

long state_elems(const wombat_weno_config *c)
{
    const int n[3] = { c->nx, c->ny, c->nz };
    long e = 8;
    for (int d = 0; d < 3; ++d) e *= n[d] + (n[d] > 1 ? 6 : 0);
    return e;
}

void make_geom(const wombat_weno_config *c, Geom &G, FaceBox F[3])
{
    const int n[3] = { c->nx, c->ny, c->nz };
    const double dl[3] = { c->dx, c->dy, c->dz };
    ww::box_geom(n, dl, G, F);
}

// Slab [k0, k0 + nk) of the box: the state geometry shifted by k0 planes
// (cells 0..nk-1 of S are planes k0.. of the box, its ghost planes the box's
// neighbouring planes) and the slab's face boxes in slab-local plane numbers:
// x and y faces on planes -1..nk (constrained transport needs one plane
// beyond the slab), z faces 0..nk.
void slab_geom(const Geom &G, int k0, int nk, Geom &S, FaceBox F[3])
{
    S = G;
    S.n[2] = nk;
    S.base = G.base + (long)k0 * G.s[2];
    for (int d = 0; d < 3; ++d) {
        FaceBox &B = F[d];
        for (int e = 0; e < 3; ++e) {
            const int n = e == 2 ? nk : G.n[e];
            if (e == d) { B.lo[e] = 0; B.cnt[e] = n + 1; }
            else if (G.act[e]) { B.lo[e] = -1; B.cnt[e] = n + 2; }
            else { B.lo[e] = 0; B.cnt[e] = 1; }
        }
        B.s[0] = 1;
        B.s[1] = B.cnt[0];
        B.s[2] = (long)B.cnt[0] * B.cnt[1];
        B.sc = (long)B.cnt[0] * B.cnt[1] * B.cnt[2];
    }
}

// The learned form's buffers (cfg.learned): the routed-step backup, the
// packed parameters, the troubled-interface queue and the decisions.
bool alloc_router(wombat_weno_t *c)
{
    if (dev_alloc(&c->backup, c->elems * c->esize) != hipSuccess) return false;
    if (dev_alloc((void **)&c->router_pk, ww::MLP_PACKED_BYTES) != hipSuccess) return false;
    long most = 1, all = 1;
    for (int d = 0; d < 3; ++d)
        if (c->G.act[d]) {
            most = std::max(most, ww::ROUTED_QUEUE_REGIONS * ww::routed_queue_capacity(d, c->F[d]));
            all += c->F[d].sc;
        }
    return dev_alloc((void **)&c->queue, sizeof(unsigned long long) * most) == hipSuccess &&
           dev_alloc((void **)&c->qcount, sizeof(int32_t) * ww::ROUTED_QUEUE_REGIONS) == hipSuccess &&
           dev_alloc((void **)&c->rmask, all) == hipSuccess;
}

void release(wombat_weno_t *c)
{
    if (!c) return;
    for (int i = 0; i < 3; ++i) { if (c->work[i]) (void)hipFree(c->work[i]); if (c->ff[i]) (void)hipFree(c->ff[i]); }
    if (c->part) (void)hipFree(c->part);
    if (c->partflag) (void)hipFree(c->partflag);
    if (c->dsmall) (void)hipFree(c->dsmall);
    if (c->hsmall) (void)hipHostFree(c->hsmall);
    if (c->nsmooth) (void)hipFree(c->nsmooth);
    if (c->backup) (void)hipFree(c->backup);
    if (c->router_pk) (void)hipFree(c->router_pk);
    if (c->queue) (void)hipFree(c->queue);
    if (c->rmask) (void)hipFree(c->rmask);
    if (c->qcount) (void)hipFree(c->qcount);
    if (c->lfg) (void)hipFree(c->lfg);
    if (c->delay) (void)hipFree(c->delay);
    if (c->cellst) (void)hipFree(c->cellst);
    for (int i = 0; i < 2; ++i) if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
}

int precheck(wombat_weno_t *c)
{
    if (!c) return fail_ctx(nullptr, WW_ERR_INVALID_ARG, "context is NULL");
    if (c->sticky) return WW_ERR_HIP;
    return WW_OK;
}

template <typename T>
int fill_ghosts_t(wombat_weno_t *c, T *u)
{
    for (int ax = 0; ax < 3; ++ax) {
        if (!c->G.act[ax]) continue;
        WW_CHECK(c, ww::launch_ghosts<T>(u, c->G, ax, c->cfg.bc, c->st));
        for (int side = 0; side < 2; ++side) {
            int face = 2 * ax + side;
            if (c->cfg.bc[face] != WW_BC_USER) continue;
            int rc = c->cfg.user_bc(c->cfg.user_bc_ctx, u, face, (void *)c->st);
            if (rc != 0) {
                char buf[96];
                snprintf(buf, sizeof buf, "user boundary hook returned %d on face %d", rc, face);
                return fail_ctx(c, WW_ERR_USER_BC, buf);
            }
        }
    }
    return WW_OK;
}

// Slab mode (cfg.slab_planes): the stage in z-slabs of `slab` planes, so that
// the face fluxes of one slab are stored instead of the whole box's, and the
// stage may write its output over its input.  Slab j reads input planes
// k0-3 .. k1+2 and writes output planes k0 .. k1-1; the next slab still reads
// planes k1-3 .. k1-1, so with out == us those three output planes go to a
// delay buffer and are copied over the input after the next slab's sweeps.
// Each face flux and cell update is computed by the same kernels and code as
// in the whole-box stage, so the results are identical bit for bit.
template <typename T>
int operator_slabs_t(wombat_weno_t *c, T *us, const T *u0, const T *acc_in, T *acc_out, T *out,
                     const ww::StageCoef &k)
{
    int rc = fill_ghosts_t<T>(c, us);
    if (rc) return rc;
    const ww::Geom &G = c->G;
    const int nz = G.n[2], kz = c->slab;
    const bool inplace = out == us;
    ww::Phys P{ c->cfg.gamma, c->cfg.eps, 1.0 / (c->cfg.gamma - 1.0) };
    T *D = (T *)c->delay;
    const long dsv = 3 * G.s[2];                          // variable stride of the delay buffer
    const long dbase = G.g[0] * G.s[0] + G.g[1] * G.s[1];  // cell (0, 0, plane 0) in it
    int pending = -1;                                     // first plane of D owed to us
    for (int k0 = 0; k0 < nz; k0 += kz) {
        const int k1 = std::min(k0 + kz, nz), nk = k1 - k0;
        ww::Geom S;
        ww::FaceBox F[3];
        slab_geom(G, k0, nk, S, F);
        for (int d = 0; d < 3; ++d)
            if (G.act[d]) WW_CHECK(c, ww::launch_sweep<T>(d, us, (T *)c->ff[d], S, F[d], P, c->cfg.weights, c->st));
        if (pending >= 0) {
            // the previous slab's last three planes: their input has been read
            for (int v = 0; v < 8; ++v)
                WW_CHECK(c, hipMemcpyAsync(us + v * G.sv + G.base - dbase + (long)pending * G.s[2], D + v * dsv,
                                           sizeof(T) * dsv, hipMemcpyDeviceToDevice, c->st));
            pending = -1;
        }
        const T *f0 = (const T *)c->ff[0], *f1 = (const T *)c->ff[1], *f2 = (const T *)c->ff[2];
        if (inplace && k1 < nz) {
            if (nk > 3) {
                ww::Geom S1 = S;
                S1.n[2] = nk - 3;
                WW_CHECK(c, ww::launch_update<T>(u0, acc_in, acc_out, out, f0, f1, f2, F, S1, k, c->st));
            }
            ww::Geom S2 = S;
            S2.n[2] = 3;
            S2.base = S.base + (long)(nk - 3) * G.s[2];
            ww::FaceBox F2[3] = { F[0], F[1], F[2] };
            for (int d = 0; d < 3; ++d) F2[d].lo[2] -= nk - 3;      // same faces, numbered from plane nk-3
            WW_CHECK(c, ww::launch_update<T>(u0, acc_in, acc_out, D, f0, f1, f2, F2, S2, k, c->st,
                                             dbase - S2.base, dsv));
            pending = k1 - 3;
        } else {
            WW_CHECK(c, ww::launch_update<T>(u0, acc_in, acc_out, out, f0, f1, f2, F, S, k, c->st));
        }
    }
    return WW_OK;
}

// Ghosts + sweeps + update (mode 0: out = L(U); mode 1: RK stage).
template <typename T>
int operator_t(wombat_weno_t *c, T *us, const T *u0, const T *acc_in, T *acc_out, T *out,
               const ww::StageCoef &k)
{
    if (c->slab) return operator_slabs_t<T>(c, us, u0, acc_in, acc_out, out, k);
    int rc;
    const bool stag = c->cellst != nullptr;
    if (stag) {
        // staggered storage: the sweeps read the cell-centred state (its
        // ghosts filled); the update advances the face slots of us's layout
        WW_CHECK(c, ww::launch_face_to_cell<T>(us, (T *)c->cellst, c->G, c->st));
        us = (T *)c->cellst;
    }
    if ((rc = fill_ghosts_t<T>(c, us))) return rc;
    ww::Phys P{ c->cfg.gamma, c->cfg.eps, 1.0 / (c->cfg.gamma - 1.0) };
    if (c->lfg) {
        // global LF speeds of the three sweeps, from this stage's state
        for (int d = 0; d < 3; ++d)
            WW_CHECK(c, ww::launch_lf_global<T>(us, c->G, d, c->cfg.gamma, c->lfg,
                                                c->lfg + ww::LF_PART_DOUBLES + 7 * d, c->st));
    }
    if (c->router && c->router_force > 0) {
        // all interfaces full: the plain sweep (same face arithmetic); no smooth ones
        const long tot = c->nsm_blocks[0] + c->nsm_blocks[1] + c->nsm_blocks[2];
        WW_CHECK(c, hipMemsetAsync(c->nsmooth, 0, sizeof(int32_t) * (tot > 0 ? tot : 1), c->st));
    }
    // with the fused x sweep the sweeps run y, z, x: the x sweep (plain or
    // routed) differences all three directions' rho, m, E fluxes and applies
    // their RK update, and the update kernel does constrained transport and
    // B only
    const bool fuse = c->fuse;
    const int order[3] = { fuse ? 1 : 0, fuse ? 2 : 1, fuse ? 0 : 2 };
    for (int m = 0; m < 3; ++m) {
        const int d = order[m];
        if (!c->G.act[d]) continue;
        if constexpr (sizeof(T) == 4) {
            if (c->router && c->router_force <= 0) {
                int32_t *ns = c->nsmooth;
                unsigned char *mk = c->rmask;
                for (int e = 0; e < d; ++e) {
                    ns += c->nsm_blocks[e];
                    if (c->G.act[e]) mk += c->F[e].sc;
                }
                const ww::XFuse<float> xf{ u0, acc_in, acc_out, out, (const float *)c->ff[1], (const float *)c->ff[2],
                                           c->F[1], c->F[2], k };
                WW_CHECK(c, ww::launch_routed_sweep(d, (const float *)us, (float *)c->ff[d], c->G, c->F[d], P,
                                                    c->router_pk, c->router_thr, c->router_force, ns,
                                                    c->queue, c->qcount, mk, c->router_reuse,
                                                    fuse && d == 0 ? &xf : nullptr, c->st));
                continue;
            }
        }
        if (c->lfg) P.ag = c->lfg + ww::LF_PART_DOUBLES + 7 * d;
        if (fuse && d == 0) {
            const ww::XFuse<T> xf{ u0, acc_in, acc_out, out, (const T *)c->ff[1], (const T *)c->ff[2],
                                   c->F[1], c->F[2], k };
            WW_CHECK(c, ww::launch_sweep_x_fused<T>(us, (T *)c->ff[0], c->G, c->F[0], P, c->cfg.weights, xf, c->st));
            continue;
        }
        WW_CHECK(c, ww::launch_sweep<T>(d, us, (T *)c->ff[d], c->G, c->F[d], P, c->cfg.weights, c->st));
    }
    ww::StageCoef kb = k;
    kb.bonly = fuse ? 1 : 0;
    kb.stag = stag ? 1 : 0;
    WW_CHECK(c, ww::launch_update<T>(u0, acc_in, acc_out, out, (const T *)c->ff[0],
                                     (const T *)c->ff[1], (const T *)c->ff[2], c->F, c->G, kb,
                                     c->st));
    return WW_OK;
}

template <typename T>
int cfl_device_t(wombat_weno_t *c, const T *u, double *d_dt, int32_t *d_flag)
{
    if (c->cellst) {     // staggered storage: wave speeds of the cell-centred field
        WW_CHECK(c, ww::launch_face_to_cell<T>(u, (T *)c->cellst, c->G, c->st));
        u = (const T *)c->cellst;
    }
    WW_CHECK(c, ww::launch_cfl<T>(u, c->G, c->cfg.gamma, c->cfg.cfl, c->part, c->partflag,
                                  c->nblk, d_dt, d_flag, c->st));
    return WW_OK;
}

// Average device time of `reps` back-to-back launches of one kernel (after
// one untimed launch), by HIP events on the context's stream.
template <typename F>
int time_launches(wombat_weno_t *c, int reps, F launch, double &ms)
{
    for (int r = 0; r <= reps; ++r) {
        if (r == 1) WW_CHECK(c, hipEventRecord(c->ev[0], c->st));
        int rc = launch();
        if (rc) return rc;
    }
    WW_CHECK(c, hipEventRecord(c->ev[1], c->st));
    WW_CHECK(c, hipEventSynchronize(c->ev[1]));
    float t = 0.0f;
    WW_CHECK(c, hipEventElapsedTime(&t, c->ev[0], c->ev[1]));
    ms = (double)t / reps;
    return WW_OK;
}

// fn(S, F) for the whole box, or for each z-slab in slab mode; stops at the
// first error.
template <typename Fn>
int for_slabs(wombat_weno_t *c, Fn fn)
{
    if (!c->slab) return fn(c->G, c->F);
    for (int k0 = 0; k0 < c->G.n[2]; k0 += c->slab) {
        ww::Geom S;
        ww::FaceBox F[3];
        slab_geom(c->G, k0, std::min(c->slab, c->G.n[2] - k0), S, F);
        int rc = fn(S, F);
        if (rc) return rc;
    }
    return WW_OK;
}

template <typename T>
int time_kernels_t(wombat_weno_t *c, T *u, int reps, double ms[7])
{
    int rc = fill_ghosts_t<T>(c, u);
    if (rc) return rc;
    ww::Phys P{ c->cfg.gamma, c->cfg.eps, 1.0 / (c->cfg.gamma - 1.0) };
    if (c->lfg)      // the global LF speeds, once, outside the timed launches
        for (int d = 0; d < 3; ++d)
            WW_CHECK(c, ww::launch_lf_global<T>(u, c->G, d, c->cfg.gamma, c->lfg,
                                                c->lfg + ww::LF_PART_DOUBLES + 7 * d, c->st));
    for (int i = 0; i < 7; ++i) ms[i] = 0.0;
    auto chk = [&](hipError_t e) { return e == hipSuccess ? (int)WW_OK : hip_fail(c, e, "timed launch"); };
    if ((rc = time_launches(c, reps, [&] {
             for (int ax = 0; ax < 3; ++ax) {
                 int r2 = chk(ww::launch_ghosts<T>(u, c->G, ax, c->cfg.bc, c->st));
                 if (r2) return r2;
             }
             return (int)WW_OK;
         }, ms[0])))
        return rc;
    // the update in the forms a step runs: the four RK4 stages (or the three
    // SSP-RK3 stages), u0 = u, acc and out in the work arrays, dt = 0 so that
    // repeated launches leave acc and out unchanged; the mean of the forms.
    // With the fused x sweep, the x sweep is timed in those forms too (the y
    // and z fluxes it reads are those of u), and the update in its B-only form.
    const bool fuse = c->fuse && !c->router;
    const T *fx = (const T *)c->ff[0], *fy = (const T *)c->ff[1], *fz = (const T *)c->ff[2];
    T *acc = (T *)c->work[c->slab ? 1 : 2], *out = (T *)c->work[0];
    const bool ssp = c->cfg.integrator == WW_SSPRK3;
    const int nform = ssp ? 3 : 4;
    auto form = [&](int s) {
        ww::StageCoef k = ssp ? ww::StageCoef{ 2, s, 0.0, 0.0, 1.0, s == 0 ? 0.0 : 0.5 }
                              : ww::StageCoef{ 1, s, 0.0, 0.0 };
        k.bonly = fuse ? 1 : 0;
        return k;
    };
    auto form_acc_in = [&](int s) {
        return ssp ? (s == 0 ? (const T *)nullptr : (const T *)c->work[1]) : (const T *)acc;
    };
    const int order[3] = { fuse ? 1 : 0, fuse ? 2 : 1, fuse ? 0 : 2 };
    for (int m = 0; m < 3; ++m) {
        const int d = order[m];
        if (!c->G.act[d]) continue;
        if (c->lfg) P.ag = c->lfg + ww::LF_PART_DOUBLES + 7 * d;
        if (fuse && d == 0) {
            double sum = 0.0;
            for (int s = 0; s < nform; ++s) {
                const ww::XFuse<T> xf{ u, form_acc_in(s), acc, out, fy, fz, c->F[1], c->F[2], form(s) };
                double t = 0.0;
                if ((rc = time_launches(c, reps, [&] {
                         return chk(ww::launch_sweep_x_fused<T>(u, (T *)c->ff[0], c->G, c->F[0], P, c->cfg.weights,
                                                                xf, c->st));
                     }, t)))
                    return rc;
                sum += t;
            }
            ms[1] = sum / nform;
            continue;
        }
        if ((rc = time_launches(c, reps, [&] {
                 return for_slabs(c, [&](const ww::Geom &S, const ww::FaceBox *F) {
                     return chk(ww::launch_sweep<T>(d, u, (T *)c->ff[d], S, F[d], P, c->cfg.weights, c->st));
                 });
             }, ms[1 + d])))
            return rc;
    }
    double sum = 0.0;
    for (int s = 0; s < nform; ++s) {
        const ww::StageCoef k = form(s);
        const T *acc_in = form_acc_in(s);
        double t = 0.0;
        if ((rc = time_launches(c, reps, [&] {
                 return for_slabs(c, [&](const ww::Geom &S, const ww::FaceBox *F) {
                     return chk(ww::launch_update<T>(u, acc_in, acc, out, fx, fy, fz, F, S, k, c->st));
                 });
             }, t)))
            return rc;
        sum += t;
    }
    ms[4] = sum / nform;
    // the CFL reduction of a step (both passes)
    if ((rc = time_launches(c, reps, [&] {
             return chk(ww::launch_cfl<T>(u, c->G, c->cfg.gamma, c->cfg.cfl, c->part, c->partflag, c->nblk,
                                          c->dsmall, c->dflag, c->st));
         }, ms[5])))
        return rc;
    // the update writing L(U) only (wombat_weno_rhs)
    ww::StageCoef k0{ 0, 0, 0.0, 0.0 };
    k0.bonly = fuse ? 1 : 0;
    return time_launches(c, reps, [&] {
        return for_slabs(c, [&](const ww::Geom &S, const ww::FaceBox *F) {
            return chk(ww::launch_update<T>(nullptr, nullptr, nullptr, out, fx, fy, fz, F, S, k0, c->st));
        });
    }, ms[6]);
}

}  // namespace

extern "C" {

int wombat_weno_abi_version(void) { return WOMBAT_WENO_ABI_VERSION; }

int64_t wombat_weno_alloc_count(void) { return (int64_t)ww::alloc_total(); }

int wombat_weno_config_default(wombat_weno_config *cfg)
{
    if (!cfg) return fail_ctx(nullptr, WW_ERR_INVALID_ARG, "config is NULL");
    memset(cfg, 0, sizeof *cfg);
    cfg->nx = cfg->ny = cfg->nz = 32;
    cfg->ng = 3;
    cfg->dx = cfg->dy = cfg->dz = 1.0 / 32.0;
    cfg->gamma = 5.0 / 3.0;
    cfg->cfl = 0.4;
    cfg->eps = 1e-6;
    cfg->precision = WW_FP64;
    return WW_OK;
}

int wombat_weno_validate_config(const wombat_weno_config *cfg)
{
    std::string why;
    int rc = validate(cfg, why);
    if (rc) return fail_ctx(nullptr, rc, why);
    return WW_OK;
}

int64_t wombat_weno_state_elems(const wombat_weno_config *cfg)
{
    std::string why;
    if (validate(cfg, why) != WW_OK) return -1;
    return state_elems(cfg);
}

int wombat_weno_init(const wombat_weno_config *cfg, wombat_weno_t **out)
{
    std::string why;
    if (!out) return fail_ctx(nullptr, WW_ERR_INVALID_ARG, "out is NULL");
    int rc = validate(cfg, why);
    if (rc) return fail_ctx(nullptr, rc, why);
    if (cfg->learned) {
        if (cfg->precision != WW_FP32_MIXED)
            return fail_ctx(nullptr, WW_ERR_UNSUPPORTED, "the learned router runs on FP32 contexts");
        if (cfg->weights != WW_WEIGHTS_JS || cfg->integrator != WW_RK4 || cfg->lf_speed != WW_LF_LOCAL)
            return fail_ctx(nullptr, WW_ERR_UNSUPPORTED,
                            "the learned router needs the WENO-JS weights, RK4 and per-stencil LF speeds");
    }
    if (cfg->slab_planes > 0) {
        if (cfg->learned || cfg->integrator != WW_RK4 || cfg->lf_speed != WW_LF_LOCAL)
            return fail_ctx(nullptr, WW_ERR_UNSUPPORTED,
                            "slab_planes runs the RK4 stages with per-stencil LF speeds, without the router");
    }
    if (cfg->b_storage == WW_B_FACE) {
        bool periodic = true;
        const int n[3] = { cfg->nx, cfg->ny, cfg->nz };
        for (int d = 0; d < 3; ++d)
            if (n[d] > 1 && (cfg->bc[2 * d] != WW_BC_PERIODIC || cfg->bc[2 * d + 1] != WW_BC_PERIODIC)) periodic = false;
        if (!periodic || cfg->slab_planes > 0 || cfg->learned)
            return fail_ctx(nullptr, WW_ERR_UNSUPPORTED,
                            "staggered B storage (WW_B_FACE) runs on periodic boxes without slab_planes or the router");
    }
    wombat_weno_t *c = new (std::nothrow) wombat_weno();
    if (!c) return fail_ctx(nullptr, WW_ERR_OOM, "host allocation failed");
    c->cfg = *cfg;
    c->slab = cfg->slab_planes > 0 ? std::min(cfg->slab_planes, cfg->nz) : 0;
    make_geom(cfg, c->G, c->F);
    c->esize = cfg->precision == WW_FP64 ? sizeof(double) : sizeof(float);
    c->elems = state_elems(cfg);
    c->st = (hipStream_t)cfg->stream;
    c->nblk = ww::cfl_blocks(c->G);
    c->fuse = !c->slab && c->G.act[0] && c->G.act[1] && c->G.act[2] && c->F[0].cnt[0] >= ww::sweep_x_fused_min_faces();
    DevGuard dg(cfg->device);
    if (!dg.ok) { delete c; return fail_ctx(nullptr, WW_ERR_HIP, "hipSetDevice failed"); }
    ww::alloc_hook_reset();
    auto oom = [&](const char *what) {
        release(c);
        delete c;
        return fail_ctx(nullptr, WW_ERR_OOM, std::string("device allocation failed: ") + what);
    };
    // slab mode: two work arrays (the stage state, updated in place, and the
    // accumulator), face fluxes of one slab and the three-plane delay buffer
    for (int i = 0; i < (c->slab ? 2 : 3); ++i)
        if (dev_alloc(&c->work[i], c->esize * c->elems) != hipSuccess) return oom("work arrays");
    {
        ww::Geom S;
        ww::FaceBox SF[3];
        if (c->slab) slab_geom(c->G, 0, c->slab, S, SF);
        for (int d = 0; d < 3; ++d)
            if (c->G.act[d] && dev_alloc(&c->ff[d], c->esize * ww::NFC * (c->slab ? SF[d].sc : c->F[d].sc)) != hipSuccess)
                return oom("face fluxes");
    }
    if (cfg->b_storage == WW_B_FACE && dev_alloc(&c->cellst, c->esize * c->elems) != hipSuccess)
        return oom("cell-centred state");
    if (c->slab) {
        const size_t db = c->esize * 8 * 3 * c->G.s[2];
        if (dev_alloc(&c->delay, db) != hipSuccess) return oom("slab delay buffer");
        if (hipMemset(c->delay, 0, db) != hipSuccess) {
            release(c);
            delete c;
            return fail_ctx(nullptr, WW_ERR_HIP, "hipMemset of the delay buffer failed");
        }
    }
    if (dev_alloc((void **)&c->part, sizeof(double) * 8 * c->nblk) != hipSuccess) return oom("partials");
    if (dev_alloc((void **)&c->partflag, sizeof(int32_t) * c->nblk) != hipSuccess) return oom("flags");
    if (dev_alloc((void **)&c->dsmall, sizeof(double) * 20) != hipSuccess) return oom("results");
    if (cfg->lf_speed == WW_LF_GLOBAL &&
        dev_alloc((void **)&c->lfg, sizeof(double) * (ww::LF_PART_DOUBLES + 21)) != hipSuccess)
        return oom("global LF speeds");
    c->dflag = (int32_t *)(c->dsmall + 16);
    if (ww::host_alloc((void **)&c->hsmall, sizeof(double) * 20) != hipSuccess) return oom("pinned host buffer");
    if (cfg->precision == WW_FP32_MIXED) {
        long tot = 0;
        for (int d = 0; d < 3; ++d) {
            c->nsm_blocks[d] = c->G.act[d] ? ww::routed_sweep_blocks(d, c->F[d]) : 0;
            tot += c->nsm_blocks[d];
        }
        if (dev_alloc((void **)&c->nsmooth, sizeof(int32_t) * (tot > 0 ? tot : 1)) != hipSuccess)
            return oom("router counters");
        if (cfg->learned && !alloc_router(c)) return oom("learned-form buffers");
    }
    for (int i = 0; i < 2; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) {
            c->ev[i] = nullptr;
            release(c);
            delete c;
            return fail_ctx(nullptr, WW_ERR_HIP, "hipEventCreate failed");
        }
    *out = c;
    return WW_OK;
}

void wombat_weno_destroy(wombat_weno_t *ctx)
{
    if (!ctx) return;
    DevGuard dg(ctx->cfg.device);
    if (!ctx->sticky) (void)hipStreamSynchronize(ctx->st);
    release(ctx);
    delete ctx;
}

const char *wombat_weno_last_error(const wombat_weno_t *ctx)
{
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

int wombat_weno_fill_ghosts(wombat_weno_t *ctx, void *d_u)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "d_u is NULL");
    DevGuard dg(ctx->cfg.device);
    if (ctx->cfg.precision == WW_FP64) return fill_ghosts_t<double>(ctx, (double *)d_u);
    return fill_ghosts_t<float>(ctx, (float *)d_u);
}

int wombat_weno_cfl_dt_device(wombat_weno_t *ctx, const void *d_u, double *d_dt, int32_t *d_flag)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u || !d_dt || !d_flag) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    DevGuard dg(ctx->cfg.device);
    if (ctx->cfg.precision == WW_FP64) return cfl_device_t<double>(ctx, (const double *)d_u, d_dt, d_flag);
    return cfl_device_t<float>(ctx, (const float *)d_u, d_dt, d_flag);
}

namespace {

// CFL step and number of non-physical cells of d_u (synchronous).
int cfl_and_count(wombat_weno_t *ctx, const void *d_u, double *dt, int32_t *bad)
{
    int rc = ctx->cfg.precision == WW_FP64
                 ? cfl_device_t<double>(ctx, (const double *)d_u, ctx->dsmall, ctx->dflag)
                 : cfl_device_t<float>(ctx, (const float *)d_u, ctx->dsmall, ctx->dflag);
    if (rc) return rc;
    WW_CHECK(ctx, hipMemcpyAsync(ctx->hsmall, ctx->dsmall, sizeof(double) * 20,
                                 hipMemcpyDeviceToHost, ctx->st));
    WW_CHECK(ctx, hipStreamSynchronize(ctx->st));
    *bad = *(int32_t *)(ctx->hsmall + 16);
    *dt = ctx->hsmall[0];
    return WW_OK;
}

int nonphysical(wombat_weno_t *ctx, int32_t bad)
{
    char buf[96];
    snprintf(buf, sizeof buf, "%d non-physical cells (rho<=0, p<=0 or non-finite)", (int)bad);
    return fail_ctx(ctx, WW_ERR_NONPHYSICAL, buf);
}

}  // namespace

int wombat_weno_cfl_dt(wombat_weno_t *ctx, const void *d_u, double *dt)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u || !dt) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    DevGuard dg(ctx->cfg.device);
    int32_t bad = 0;
    double d = 0.0;
    if ((rc = cfl_and_count(ctx, d_u, &d, &bad))) return rc;
    if (bad) return nonphysical(ctx, bad);
    *dt = d;
    return WW_OK;
}

int wombat_weno_rhs(wombat_weno_t *ctx, void *d_u, void *d_dudt)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u || !d_dudt) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    if (d_u == d_dudt) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "d_dudt must not alias d_u");
    DevGuard dg(ctx->cfg.device);
    ww::StageCoef k{ 0, 0, 0.0, 0.0 };
    if (ctx->cfg.precision == WW_FP64)
        return operator_t<double>(ctx, (double *)d_u, nullptr, nullptr, nullptr, (double *)d_dudt, k);
    return operator_t<float>(ctx, (float *)d_u, nullptr, nullptr, nullptr, (float *)d_dudt, k);
}

int wombat_weno_stage(wombat_weno_t *ctx, int s, double dt, const void *d_u0, void *d_us_in,
                      void *d_acc, void *d_us_out)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (ctx->cfg.integrator != WW_RK4)
        return fail_ctx(ctx, WW_ERR_UNSUPPORTED, "wombat_weno_stage runs the classical RK4 stages");
    if (s < 0 || s > 3) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "stage must be 0..3");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (!d_us_in || !d_acc || !d_us_out || (s < 3 && !d_u0))
        return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    if (d_us_out == d_us_in && !ctx->slab)
        return fail_ctx(ctx, WW_ERR_INVALID_ARG, "d_us_out must not alias d_us_in (except with slab_planes)");
    if (d_acc == d_us_in || d_acc == d_us_out || (s < 3 && d_acc == d_u0))
        return fail_ctx(ctx, WW_ERR_INVALID_ARG, "d_acc must not alias the other arrays");
    DevGuard dg(ctx->cfg.device);
    static const double bw[4] = { 1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 0.0 };
    static const double cw[4] = { 0.5, 0.5, 1.0, 1.0 / 6.0 };
    ww::StageCoef k{ 1, s, bw[s] * dt, cw[s] * dt };
    if (ctx->cfg.precision == WW_FP64)
        return operator_t<double>(ctx, (double *)d_us_in, (const double *)d_u0, (const double *)d_acc,
                                  (double *)d_acc, (double *)d_us_out, k);
    return operator_t<float>(ctx, (float *)d_us_in, (const float *)d_u0, (const float *)d_acc,
                             (float *)d_acc, (float *)d_us_out, k);
}

namespace {

// The four stages of a step.  With routing on, the network is evaluated at
// the first stage and its decisions reused for the other three.
int rk4_stages(wombat_weno_t *ctx, void *d_u, double dt)
{
    int rc;
    if (ctx->slab) {
        // the stage state A is updated in place; acc accumulates
        void *A = ctx->work[0], *acc = ctx->work[1];
        if (!(rc = wombat_weno_stage(ctx, 0, dt, d_u, d_u, acc, A)) &&
            !(rc = wombat_weno_stage(ctx, 1, dt, d_u, A, acc, A)) &&
            !(rc = wombat_weno_stage(ctx, 2, dt, d_u, A, acc, A)))
            rc = wombat_weno_stage(ctx, 3, dt, d_u, A, acc, d_u);
        return rc;
    }
    void *A = ctx->work[0], *B = ctx->work[1], *acc = ctx->work[2];
    ctx->router_reuse = 0;
    if ((rc = wombat_weno_stage(ctx, 0, dt, d_u, d_u, acc, A))) return rc;
    ctx->router_reuse = ctx->router ? 1 : 0;
    if (!(rc = wombat_weno_stage(ctx, 1, dt, d_u, A, acc, B)) &&
        !(rc = wombat_weno_stage(ctx, 2, dt, d_u, B, acc, A)))
        rc = wombat_weno_stage(ctx, 3, dt, d_u, A, acc, d_u);
    ctx->router_reuse = 0;
    return rc;
}

// The three stages of an SSP-RK3 step (Shu & Osher 1988); each writes
// out = a0 u^n + a1 us + c dt L(us) (the update kernel's mode 2).
int ssprk3_stages(wombat_weno_t *ctx, void *d_u, double dt)
{
    void *A = ctx->work[0], *B = ctx->work[1];
    const ww::StageCoef k0{ 2, 0, 0.0, dt, 1.0, 0.0 };
    const ww::StageCoef k1{ 2, 1, 0.0, 0.25 * dt, 0.75, 0.25 };
    const ww::StageCoef k2{ 2, 2, 0.0, 2.0 / 3.0 * dt, 1.0 / 3.0, 2.0 / 3.0 };
    DevGuard dg(ctx->cfg.device);
    int rc;
    if (ctx->cfg.precision == WW_FP64) {
        double *u = (double *)d_u, *a = (double *)A, *b = (double *)B;
        if (!(rc = operator_t<double>(ctx, u, u, nullptr, nullptr, a, k0)) &&
            !(rc = operator_t<double>(ctx, a, u, a, nullptr, b, k1)))
            rc = operator_t<double>(ctx, b, u, b, nullptr, u, k2);
        return rc;
    }
    float *u = (float *)d_u, *a = (float *)A, *b = (float *)B;
    if (!(rc = operator_t<float>(ctx, u, u, nullptr, nullptr, a, k0)) &&
        !(rc = operator_t<float>(ctx, a, u, a, nullptr, b, k1)))
        rc = operator_t<float>(ctx, b, u, b, nullptr, u, k2);
    return rc;
}

}  // namespace

int wombat_weno_step(wombat_weno_t *ctx, void *d_u, double dt, double *dt_used)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "d_u is NULL");
    if (!std::isfinite(dt)) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "dt must be finite");
    if (dt <= 0.0) {
        rc = wombat_weno_cfl_dt(ctx, d_u, &dt);
        if (rc) return rc;
    }
    // a routed step keeps u^n; if it leaves a non-physical cell the step is
    // redone from u^n with full characteristic WENO everywhere
    const bool guard = ctx->router && ctx->router_force == 0;
    if (guard) {
        DevGuard dg(ctx->cfg.device);
        WW_CHECK(ctx, hipMemcpyAsync(ctx->backup, d_u, ctx->elems * ctx->esize, hipMemcpyDeviceToDevice,
                                     ctx->st));
    }
    if (ctx->cfg.integrator == WW_SSPRK3) {
        if ((rc = ssprk3_stages(ctx, d_u, dt))) return rc;
    } else if ((rc = rk4_stages(ctx, d_u, dt))) {
        return rc;
    }
    if (guard) {
        DevGuard dg(ctx->cfg.device);
        int32_t bad = 0;
        double unused;
        if ((rc = cfl_and_count(ctx, d_u, &unused, &bad))) return rc;
        if (bad) {
            WW_CHECK(ctx, hipMemcpyAsync(d_u, ctx->backup, ctx->elems * ctx->esize,
                                         hipMemcpyDeviceToDevice, ctx->st));
            ctx->router_force = 1;
            rc = rk4_stages(ctx, d_u, dt);
            ctx->router_force = 0;
            if (rc) return rc;
            ++ctx->fallbacks;
        }
    }
    if (dt_used) *dt_used = dt;
    return WW_OK;
}

int wombat_weno_sums(wombat_weno_t *ctx, const void *d_u, double out[8])
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u || !out) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    DevGuard dg(ctx->cfg.device);
    if (ctx->cfg.precision == WW_FP64)
        WW_CHECK(ctx, ww::launch_sums<double>((const double *)d_u, ctx->G, ctx->part, ctx->nblk,
                                              ctx->dsmall + 1, ctx->st));
    else
        WW_CHECK(ctx, ww::launch_sums<float>((const float *)d_u, ctx->G, ctx->part, ctx->nblk,
                                             ctx->dsmall + 1, ctx->st));
    WW_CHECK(ctx, hipMemcpyAsync(ctx->hsmall, ctx->dsmall, sizeof(double) * 20,
                                 hipMemcpyDeviceToHost, ctx->st));
    WW_CHECK(ctx, hipStreamSynchronize(ctx->st));
    for (int v = 0; v < 8; ++v) out[v] = ctx->hsmall[1 + v];
    return WW_OK;
}

int wombat_weno_divb(wombat_weno_t *ctx, void *d_u, double *max_abs, double *l1)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u || !max_abs || !l1) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    if ((rc = wombat_weno_fill_ghosts(ctx, d_u))) return rc;
    DevGuard dg(ctx->cfg.device);
    if (ctx->cellst && ctx->cfg.precision == WW_FP64)
        WW_CHECK(ctx, ww::launch_divb_face<double>((const double *)d_u, ctx->G, ctx->part, ctx->nblk,
                                                   ctx->dsmall + 1, ctx->st));
    else if (ctx->cellst)
        WW_CHECK(ctx, ww::launch_divb_face<float>((const float *)d_u, ctx->G, ctx->part, ctx->nblk,
                                                  ctx->dsmall + 1, ctx->st));
    else if (ctx->cfg.precision == WW_FP64)
        WW_CHECK(ctx, ww::launch_divb<double>((const double *)d_u, ctx->G, ctx->part, ctx->nblk,
                                              ctx->dsmall + 1, ctx->st));
    else
        WW_CHECK(ctx, ww::launch_divb<float>((const float *)d_u, ctx->G, ctx->part, ctx->nblk,
                                             ctx->dsmall + 1, ctx->st));
    WW_CHECK(ctx, hipMemcpyAsync(ctx->hsmall, ctx->dsmall, sizeof(double) * 20,
                                 hipMemcpyDeviceToHost, ctx->st));
    WW_CHECK(ctx, hipStreamSynchronize(ctx->st));
    *max_abs = ctx->hsmall[1];
    *l1 = ctx->hsmall[2];
    return WW_OK;
}

int wombat_weno_time_kernels(wombat_weno_t *ctx, void *d_u, int reps, double ms[7])
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u || !ms) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    if (reps < 1 || reps > 1000) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "reps must be in 1..1000");
    DevGuard dg(ctx->cfg.device);
    if (ctx->cfg.precision == WW_FP64) return time_kernels_t<double>(ctx, (double *)d_u, reps, ms);
    return time_kernels_t<float>(ctx, (float *)d_u, reps, ms);
}

int wombat_weno_set_router(wombat_weno_t *ctx, const float *d_theta, double threshold, int mode)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (ctx->cfg.precision != WW_FP32_MIXED)
        return fail_ctx(ctx, WW_ERR_UNSUPPORTED, "the learned router runs on FP32 contexts");
    if (ctx->cfg.weights != WW_WEIGHTS_JS)
        return fail_ctx(ctx, WW_ERR_UNSUPPORTED, "the learned router routes to the WENO-JS flux only");
    if (ctx->cfg.integrator != WW_RK4)
        return fail_ctx(ctx, WW_ERR_UNSUPPORTED, "the learned router runs with the RK4 step only");
    if (ctx->cfg.lf_speed != WW_LF_LOCAL)
        return fail_ctx(ctx, WW_ERR_UNSUPPORTED, "the learned router uses the per-stencil LF speeds only");
    if (!d_theta) { ctx->router = 0; return WW_OK; }
    if (!(threshold > 0.0 && threshold < 1.0)) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "threshold must be in (0, 1)");
    if (mode < -1 || mode > 1) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "mode must be -1, 0 or 1");
    if (!ctx->router_pk)
        return fail_ctx(ctx, WW_ERR_STATE, "the context was created without cfg.learned = 1 (the learned "
                                           "form's buffers are allocated by wombat_weno_init)");
    DevGuard dg(ctx->cfg.device);
    WW_CHECK(ctx, ww::launch_pack_mlp(d_theta, ctx->router_pk, ctx->st));
    ctx->router = 1;
    ctx->router_thr = (float)std::log(threshold / (1.0 - threshold));
    ctx->router_force = mode;
    return WW_OK;
}

int wombat_weno_router_stats(wombat_weno_t *ctx, int64_t *smooth, int64_t *total, int64_t *fallbacks)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!smooth || !total) return fail_ctx(ctx, WW_ERR_INVALID_ARG, "NULL pointer");
    if (!ctx->nsmooth) return fail_ctx(ctx, WW_ERR_UNSUPPORTED, "no router counters (FP64 context)");
    DevGuard dg(ctx->cfg.device);
    long tot = ctx->nsm_blocks[0] + ctx->nsm_blocks[1] + ctx->nsm_blocks[2];
    std::string buf;
    int32_t *h = nullptr;
    WW_CHECK(ctx, hipStreamSynchronize(ctx->st));
    h = (int32_t *)malloc(sizeof(int32_t) * (tot > 0 ? tot : 1));
    if (!h) return fail_ctx(ctx, WW_ERR_OOM, "host allocation failed");
    hipError_t e = hipMemcpy(h, ctx->nsmooth, sizeof(int32_t) * tot, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { free(h); return hip_fail(ctx, e, "hipMemcpy router counters"); }
    int64_t s = 0;
    for (long i = 0; i < tot; ++i) s += h[i];
    free(h);
    int64_t faces = 0;
    for (int d = 0; d < 3; ++d) if (ctx->G.act[d]) faces += ctx->F[d].sc;
    *smooth = s;
    *total = faces;
    if (fallbacks) *fallbacks = ctx->fallbacks;
    return WW_OK;
}

int wombat_weno_router_sample(wombat_weno_t *ctx, void *d_u, const int32_t *d_where, int n,
                              float *d_X, float *d_dev, float *d_excess)
{
    int rc = precheck(ctx);
    if (rc) return rc;
    if (!d_u || !d_where || !d_X || !d_dev || !d_excess || n < 1)
        return fail_ctx(ctx, WW_ERR_INVALID_ARG, "bad argument");
    if ((rc = wombat_weno_fill_ghosts(ctx, d_u))) return rc;
    DevGuard dg(ctx->cfg.device);
    ww::Phys P{ ctx->cfg.gamma, ctx->cfg.eps, 1.0 / (ctx->cfg.gamma - 1.0) };
    if (ctx->cfg.precision == WW_FP64)
        WW_CHECK(ctx, ww::launch_router_sample<double>((const double *)d_u, ctx->G, P, d_where, n, d_X, d_dev, d_excess, ctx->st));
    else
        WW_CHECK(ctx, ww::launch_router_sample<float>((const float *)d_u, ctx->G, P, d_where, n, d_X, d_dev, d_excess, ctx->st));
    return WW_OK;
}

int wombat_mlp_forward(void *stream, const float *d_theta, const float *d_X, int n, float *d_logit)
{
    if (!d_theta || !d_X || !d_logit || n < 1) return fail_ctx(nullptr, WW_ERR_INVALID_ARG, "bad argument");
    hipError_t e = ww::launch_mlp_infer(d_theta, d_X, n, d_logit, (hipStream_t)stream);
    return e == hipSuccess ? WW_OK : hip_fail(nullptr, e, "mlp forward");
}

int64_t wombat_mlp_grad_workspace(int n)
{
    return n < 1 ? -1 : (int64_t)ww::mlp_grad_blocks(n) * (ww::NPARAM + 1);
}

int wombat_mlp_grad(void *stream, const float *d_theta, const float *d_X, const float *d_t, int n,
                    float *d_work, float *d_grad, float *d_loss)
{
    if (!d_theta || !d_X || !d_t || !d_work || !d_grad || n < 1)
        return fail_ctx(nullptr, WW_ERR_INVALID_ARG, "bad argument");
    hipError_t e = ww::launch_mlp_grad(d_theta, d_X, d_t, n, d_work, d_grad, d_loss, (hipStream_t)stream);
    return e == hipSuccess ? WW_OK : hip_fail(nullptr, e, "mlp grad");
}

int wombat_mlp_adam(void *stream, float *d_theta, float *d_m, float *d_v, const float *d_grad,
                    int step, float lr, float beta1, float beta2, float eps)
{
    if (!d_theta || !d_m || !d_v || !d_grad || step < 1 || !(lr > 0.f))
        return fail_ctx(nullptr, WW_ERR_INVALID_ARG, "bad argument");
    hipError_t e = ww::launch_mlp_adam(d_theta, d_m, d_v, d_grad, step, lr, beta1, beta2, eps, (hipStream_t)stream);
    return e == hipSuccess ? WW_OK : hip_fail(nullptr, e, "mlp adam");
}

int wombat_mlp_param_count(void) { return ww::NPARAM; }

}  // extern "C"
