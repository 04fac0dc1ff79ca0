// ww_noalloc.hip -- wombat_weno_rhs_noalloc: the right-hand side of
// wombat_weno_rhs without a context and without any allocation, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops).  The face fluxes of the three sweeps (and, with global LF
// speeds, their partial maxima) go to one file-scope device array of fixed
// size; each GPU the library runs on holds its own copy until the process
// ends.  The kernels are those of the context path (same launches, same
// results bit for bit).
#include "ww_internal.h"

#include <mutex>

namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;    // 64 MiB per device
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Device address of `scratch` per device ordinal, taken once per device with
// that device current.  In host code the array's name is only a stand-in for
// the symbol; kernels get this address.
void *g_scratch[MAX_DEVICES];
std::mutex g_mu;

hipError_t scratch_ptr(int dev, void **p)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = q;
    }
    *p = g_scratch[dev];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int fail(int code, const std::string &msg)
{
    ww::set_global_error(msg);
    return code;
}

int hipfail(hipError_t e, const char *what)
{
    return fail(WW_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
int rhs_t(const wombat_weno_config *cfg, const ww::Geom &G, const ww::FaceBox (&F)[3], char *buf, T *u,
          T *dudt)
{
    hipStream_t st = (hipStream_t)cfg->stream;
    // ghost zones, axis by axis, then the user faces of that axis (Sec. 2.2)
    for (int ax = 0; ax < 3; ++ax) {
        if (!G.act[ax]) continue;
        hipError_t e = ww::launch_ghosts<T>(u, G, ax, cfg->bc, st);
        if (e != hipSuccess) return hipfail(e, "ghost fill");
        for (int side = 0; side < 2; ++side) {
            const int face = 2 * ax + side;
            if (cfg->bc[face] != WW_BC_USER) continue;
            const int rc = cfg->user_bc(cfg->user_bc_ctx, u, face, (void *)st);
            if (rc != 0)
                return fail(WW_ERR_USER_BC, "user boundary hook returned " + std::to_string(rc) + " on face " +
                                                std::to_string(face));
        }
    }
    T *ff[3] = { nullptr, nullptr, nullptr };
    size_t off = 0;
    for (int d = 0; d < 3; ++d) {
        if (!G.act[d]) continue;
        ff[d] = (T *)(buf + off);
        off += align256(sizeof(T) * ww::NFC * F[d].sc);
    }
    double *lfg = cfg->lf_speed == WW_LF_GLOBAL ? (double *)(buf + off) : nullptr;
    ww::Phys P{ cfg->gamma, cfg->eps, 1.0 / (cfg->gamma - 1.0) };
    for (int d = 0; d < 3; ++d) {
        if (!G.act[d]) continue;
        if (lfg) {
            hipError_t e = ww::launch_lf_global<T>(u, G, d, cfg->gamma, lfg, lfg + ww::LF_PART_DOUBLES + 7 * d, st);
            if (e != hipSuccess) return hipfail(e, "global LF speeds");
            P.ag = lfg + ww::LF_PART_DOUBLES + 7 * d;
        }
        hipError_t e = ww::launch_sweep<T>(d, u, ff[d], G, F[d], P, cfg->weights, st);
        if (e != hipSuccess) return hipfail(e, "sweep");
    }
    const ww::StageCoef k{ 0, 0, 0.0, 0.0 };
    hipError_t e = ww::launch_update<T>(nullptr, nullptr, nullptr, dudt, ff[0], ff[1], ff[2], F, G, k, st);
    return e == hipSuccess ? (int)WW_OK : hipfail(e, "update");
}

}  // namespace

extern "C" {

int wombat_weno_rhs_noalloc(const wombat_weno_config *cfg, void *d_u, void *d_dudt)
{
    std::string why;
    int rc = ww::validate_config(cfg, why);
    if (rc) return fail(rc, why);
    if (!d_u || !d_dudt) return fail(WW_ERR_INVALID_ARG, "NULL pointer");
    if (d_u == d_dudt) return fail(WW_ERR_INVALID_ARG, "d_dudt must not alias d_u");
    if (cfg->learned) return fail(WW_ERR_UNSUPPORTED, "the learned router needs a context");
    if (cfg->b_storage != WW_B_CELL || cfg->slab_planes != 0)
        return fail(WW_ERR_UNSUPPORTED, "staggered B storage and slab_planes need a context");
    if (cfg->device >= MAX_DEVICES) return fail(WW_ERR_UNSUPPORTED, "device ordinal beyond 63");
    ww::Geom G;
    ww::FaceBox F[3];
    const int n[3] = { cfg->nx, cfg->ny, cfg->nz };
    const double dl[3] = { cfg->dx, cfg->dy, cfg->dz };
    ww::box_geom(n, dl, G, F);
    const size_t es = cfg->precision == WW_FP64 ? sizeof(double) : sizeof(float);
    size_t need = 0;
    for (int d = 0; d < 3; ++d)
        if (G.act[d]) need += align256(es * ww::NFC * F[d].sc);
    if (cfg->lf_speed == WW_LF_GLOBAL) need += sizeof(double) * (ww::LF_PART_DOUBLES + 21);
    if (need > SCRATCH_BYTES)
        return fail(WW_ERR_INVALID_ARG, "box too large for the no-allocation scratch: needs " + std::to_string(need) +
                                            " bytes, the maximum is " + std::to_string(SCRATCH_BYTES));
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != cfg->device) {
        hipError_t e = hipSetDevice(cfg->device);
        if (e != hipSuccess) return hipfail(e, "hipSetDevice");
    }
    void *buf = nullptr;
    hipError_t e = scratch_ptr(cfg->device, &buf);
    if (e != hipSuccess) rc = hipfail(e, "hipGetSymbolAddress(scratch)");
    else if (cfg->precision == WW_FP64) rc = rhs_t<double>(cfg, G, F, (char *)buf, (double *)d_u, (double *)d_dudt);
    else rc = rhs_t<float>(cfg, G, F, (char *)buf, (float *)d_u, (float *)d_dudt);
    if (prev >= 0 && prev != cfg->device) (void)hipSetDevice(prev);
    return rc;
}

}  // extern "C"
