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
// marching in k.  The z-face fluxes and the EMFs of the upper z-level are
// carried to the next cell; the EMF of every edge is formed exactly as in
// emf() (same operands, same order), so results equal the general kernel's.
// Hardware block b runs on XCD b % 8; blocks are renumbered so that each XCD
// owns a contiguous range of tiles (neighbouring rows share its L2).
template <typename T>
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

    const T *FX = a.ff[0], *FY = a.ff[1], *FZ = a.ff[2];
    const FaceBox &BX = a.fb[0], &BY = a.fb[1], &BZ = a.fb[2];
    const long sx = BX.sc, sy = BY.sc, sz = BZ.sc;
    const T idx = T(G.idl[0]), idy = T(G.idl[1]), idz = T(G.idl[2]);
    const T q = T(0.25);
    // E_y(fz, fx, j) = 1/4[-FZ4(fx-1,j,fz) - FZ4(fx,j,fz) + FX5(fx,j,fz-1) + FX5(fx,j,fz)]
    // E_x(fy, fz, i) = 1/4[-FY4(i,fy,fz-1) - FY4(i,fy,fz) + FZ5(i,fy-1,fz) + FZ5(i,fy,fz)]
    // E_z(fx, fy, k) = 1/4[-FX4(fx,fy-1,k) - FX4(fx,fy,k) + FY5(fx-1,fy,k) + FY5(fx,fy,k)]
    auto ey = [&](int fz, int fx, T x5lo, T x5hi) {
        T t = -FZ[4 * sz + BZ.idx(fx - 1, j, fz)];
        t -= FZ[4 * sz + BZ.idx(fx, j, fz)];
        t += x5lo;
        t += x5hi;
        return q * t;
    };
    auto ex = [&](int fy, int fz, T y4lo, T y4hi) {
        T t = -y4lo;
        t -= y4hi;
        t += FZ[5 * sz + BZ.idx(i, fy - 1, fz)];
        t += FZ[5 * sz + BZ.idx(i, fy, fz)];
        return q * t;
    };
    auto ez = [&](int fx, int fy, int k) {
        T t = -FX[4 * sx + BX.idx(fx, fy - 1, k)];
        t -= FX[4 * sx + BX.idx(fx, fy, k)];
        t += FY[5 * sy + BY.idx(fx - 1, fy, k)];
        t += FY[5 * sy + BY.idx(fx, fy, k)];
        return q * t;
    };

    // carried values at the lower z-level k (face fz = k)
    T x5lo0 = FX[5 * sx + BX.idx(i, j, k0 - 1)], x5lo1 = FX[5 * sx + BX.idx(i + 1, j, k0 - 1)];
    T x5c0 = FX[5 * sx + BX.idx(i, j, k0)], x5c1 = FX[5 * sx + BX.idx(i + 1, j, k0)];
    T y4lo0 = FY[4 * sy + BY.idx(i, j, k0 - 1)], y4lo1 = FY[4 * sy + BY.idx(i, j + 1, k0 - 1)];
    T y4c0 = FY[4 * sy + BY.idx(i, j, k0)], y4c1 = FY[4 * sy + BY.idx(i, j + 1, k0)];
    T Ey0 = ey(k0, i, x5lo0, x5c0), Ey1 = ey(k0, i + 1, x5lo1, x5c1);     // E_y(k, i|i+1, j)
    T Ex0 = ex(j, k0, y4lo0, y4c0), Ex1 = ex(j + 1, k0, y4lo1, y4c1);     // E_x(j|j+1, k, i)
    const int hs[5] = { 0, 1, 2, 3, 6 }, hv[5] = { 0, 1, 2, 3, 7 };
    T fzlo[5];
#pragma unroll
    for (int h = 0; h < 5; ++h) fzlo[h] = FZ[hs[h] * sz + BZ.idx(i, j, k0)];

    for (int k = k0; k < k1; ++k) {
        const long id = G.base + i * G.s[0] + j * G.s[1] + (long)k * G.s[2];
        T L[8];
        T fzhi[5];
#pragma unroll
        for (int h = 0; h < 5; ++h) {
            T acc = T(0);
            T fr = FX[hs[h] * sx + BX.idx(i + 1, j, k)], fl = FX[hs[h] * sx + BX.idx(i, j, k)];
            acc -= (fr - fl) * idx;
            fr = FY[hs[h] * sy + BY.idx(i, j + 1, k)];
            fl = FY[hs[h] * sy + BY.idx(i, j, k)];
            acc -= (fr - fl) * idy;
            fzhi[h] = FZ[hs[h] * sz + BZ.idx(i, j, k + 1)];
            acc -= (fzhi[h] - fzlo[h]) * idz;
            L[hv[h]] = acc;
        }
        // EMFs of this cell's edges
        const T x5h0 = FX[5 * sx + BX.idx(i, j, k + 1)], x5h1 = FX[5 * sx + BX.idx(i + 1, j, k + 1)];
        const T y4h0 = FY[4 * sy + BY.idx(i, j, k + 1)], y4h1 = FY[4 * sy + BY.idx(i, j + 1, k + 1)];
        const T Ey2 = ey(k + 1, i, x5c0, x5h0), Ey3 = ey(k + 1, i + 1, x5c1, x5h1);  // E_y(k+1, i|i+1, j)
        const T Ex2 = ex(j, k + 1, y4c0, y4h0), Ex3 = ex(j + 1, k + 1, y4c1, y4h1);  // E_x(j|j+1, k+1, i)
        const T Ez00 = ez(i, j, k), Ez10 = ez(i + 1, j, k), Ez01 = ez(i, j + 1, k), Ez11 = ez(i + 1, j + 1, k);
        // face updates (same operation order as face_bdot)
        T r;
        T bxl, bxr, byl, byr, bzl, bzr;
        r = T(0); r -= (Ez01 - Ez00) * idy; r += (Ey2 - Ey0) * idz; bxl = r;
        r = T(0); r -= (Ez11 - Ez10) * idy; r += (Ey3 - Ey1) * idz; bxr = r;
        r = T(0); r -= (Ex2 - Ex0) * idz; r += (Ez10 - Ez00) * idx; byl = r;
        r = T(0); r -= (Ex3 - Ex1) * idz; r += (Ez11 - Ez01) * idx; byr = r;
        r = T(0); r -= (Ey1 - Ey0) * idx; r += (Ex1 - Ex0) * idy; bzl = r;
        r = T(0); r -= (Ey3 - Ey2) * idx; r += (Ex3 - Ex2) * idy; bzr = r;
        L[4] = T(0.5) * (bxl + bxr);
        L[5] = T(0.5) * (byl + byr);
        L[6] = T(0.5) * (bzl + bzr);
        rk_store(a, id, L);
        // carry to level k+1
        Ey0 = Ey2; Ey1 = Ey3; Ex0 = Ex2; Ex1 = Ex3;
        x5c0 = x5h0; x5c1 = x5h1; y4c0 = y4h0; y4c1 = y4h1;
#pragma unroll
        for (int h = 0; h < 5; ++h) fzlo[h] = fzhi[h];
    }
}

}  // namespace

template <typename T>
hipError_t launch_update(const T *u0, const T *acc_in, T *acc_out, T *out, const T *fx,
                         const T *fy, const T *fz, const FaceBox *F, const Geom &G,
                         const StageCoef &c, hipStream_t st)
{
    UpdArgs<T> a;
    a.u0 = u0; a.acc_in = acc_in; a.acc_out = acc_out; a.out = out;
    a.ff[0] = fx; a.ff[1] = fy; a.ff[2] = fz;
    for (int d = 0; d < 3; ++d) a.fb[d] = F[d];
    a.G = G;
    a.c = c;
    if (G.act[0] && G.act[1] && G.act[2]) {
        int ntx = (G.n[0] + MX_TX - 1) / MX_TX, nty = (G.n[1] + MX_TY - 1) / MX_TY,
            ntz = (G.n[2] + MX_KZ - 1) / MX_KZ;
        int nb = ntx * nty * ntz, per = (nb + NXCD - 1) / NXCD;
        hipLaunchKernelGGL((update_march_kernel<T>), dim3(per * NXCD), dim3(MX_TX, MX_TY), 0, st, a,
                           ntx, nty, ntz, per);
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
                                          hipStream_t);
template hipError_t launch_update<float>(const float *, const float *, float *, float *,
                                         const float *, const float *, const float *,
                                         const FaceBox *, const Geom &, const StageCoef &,
                                         hipStream_t);

}  // namespace ww
