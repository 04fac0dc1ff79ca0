// ww_update.hip -- launchers of the flux-difference / CT / RK update kernels
// (device code in ww_update_dev.h).
#include "ww_update_dev.h"

namespace ww {
namespace {

using up::UpdArgs;
using up::rk_store;

template <typename T>
__global__ __launch_bounds__(256) void update_kernel(UpdArgs<T> a)
{
    const Geom &G = a.G;
    const long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell) return;
    int pos[3];
    pos[0] = (int)(t % G.n[0]);
    pos[1] = (int)((t / G.n[0]) % G.n[1]);
    pos[2] = (int)(t / ((long)G.n[0] * G.n[1]));
    up::update_cell(a, pos);
}

constexpr int MX_TX = 64, MX_TY = 4, MX_KZ = 16;   // march tile: x lanes, y rows, z cells
constexpr int NXCD = 8;                              // MI355X: 8 XCDs, blocks dealt round-robin

// Three active axes: one thread per (i, j) column segment of MX_KZ cells,
// marching in k (up::march_column).  Hardware block b runs on XCD b % 8;
// blocks are renumbered so that each XCD owns a contiguous range of tiles
// (neighbouring rows share its L2).
template <typename T, bool BONLY, bool STAG>
__global__ __launch_bounds__(256) void update_march_kernel(UpdArgs<T> a, int ntx, int nty, int ntz,
                                                           int per_xcd)
{
    const Geom &G = a.G;
    const int hb = blockIdx.x;
    const int lb = (hb % NXCD) * per_xcd + hb / NXCD;
    if (lb >= ntx * nty * ntz) return;
    const int bx = lb % ntx, by = (lb / ntx) % nty, bz = lb / (ntx * nty);
    const int i = bx * MX_TX + threadIdx.x, j = by * MX_TY + threadIdx.y;
    if (i >= G.n[0] || j >= G.n[1]) return;
    const int k0 = bz * MX_KZ, k1 = min(k0 + MX_KZ, G.n[2]);
    up::march_column<T, BONLY, STAG>(a, i, j, k0, k1);
}

}  // namespace

template <typename T>
hipError_t launch_update(const T *u0, const T *acc_in, T *acc_out, T *out, const T *fx,
                         const T *fy, const T *fz, const FaceBox *F, const Geom &G,
                         const StageCoef &c, hipStream_t st, long odelta, long osv)
{
    UpdArgs<T> a;
    a.odelta = odelta;
    a.osv = osv > 0 ? osv : G.sv;
    a.u0 = u0; a.acc_in = acc_in; a.acc_out = acc_out; a.out = out;
    a.ff[0] = fx; a.ff[1] = fy; a.ff[2] = fz;
    for (int d = 0; d < 3; ++d) a.fb[d] = F[d];
    a.G = G;
    a.c = c;
    if (G.act[0] && G.act[1] && G.act[2]) {
        int ntx = (G.n[0] + MX_TX - 1) / MX_TX, nty = (G.n[1] + MX_TY - 1) / MX_TY,
            ntz = (G.n[2] + MX_KZ - 1) / MX_KZ;
        int nb = ntx * nty * ntz, per = (nb + NXCD - 1) / NXCD;
        const dim3 grd(per * NXCD), blk(MX_TX, MX_TY);
        if (c.bonly && c.stag)
            hipLaunchKernelGGL((update_march_kernel<T, true, true>), grd, blk, 0, st, a, ntx, nty, ntz, per);
        else if (c.bonly)
            hipLaunchKernelGGL((update_march_kernel<T, true, false>), grd, blk, 0, st, a, ntx, nty, ntz, per);
        else if (c.stag)
            hipLaunchKernelGGL((update_march_kernel<T, false, true>), grd, blk, 0, st, a, ntx, nty, ntz, per);
        else
            hipLaunchKernelGGL((update_march_kernel<T, false, false>), grd, blk, 0, st, a, ntx, nty, ntz, per);
        return hipGetLastError();
    }
    long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    dim3 grd((unsigned)((ncell + 255) / 256));
    hipLaunchKernelGGL((update_kernel<T>), grd, dim3(256), 0, st, a);
    return hipGetLastError();
}

template hipError_t launch_update<double>(const double *, const double *, double *, double *,
                                          const double *, const double *, const double *,
                                          const FaceBox *, const Geom &, const StageCoef &,
                                          hipStream_t, long, long);
template hipError_t launch_update<float>(const float *, const float *, float *, float *,
                                         const float *, const float *, const float *,
                                         const FaceBox *, const Geom &, const StageCoef &,
                                         hipStream_t, long, long);

}  // namespace ww
