// ww_update_dev.h -- device code of the flux difference, constrained
// transport and RK update, shared by the single-box and batched kernels.
//
// One thread per interior cell (arXiv:1808.10633, Sec. 2.1-2.2):
//   L(U) for rho, m, E = -sum_d (F_d(i+1/2) - F_d(i-1/2)) / dx_d, x then y then z;
//   L(U) for B from constrained transport: edge EMFs are the mean of the four
//   adjacent face fluxes of the transverse field (the p-flux of B_q is -E_c,
//   the q-flux of B_p is +E_c for cyclic (p, q, c)); the staggered normal
//   field of each face advances by -(curl E)_n, and the cell-centred field by
//   the mean of its two faces.  On an inactive axis the missing derivative
//   vanishes and the EMF is the single available estimate.
//   Then the low-storage classical RK4 update of the stage, or a stage of
//   SSP-RK3 (the integrator ablation).
#pragma once
#include "ww_internal.h"

namespace ww {
namespace up {

template <typename T>
struct UpdArgs {
    const T *u0;
    const T *acc_in;
    T *acc_out;
    T *out;
    const T *ff[3];
    FaceBox fb[3];
    Geom G;
    StageCoef c;
    long odelta;       // out[v] of the cell at index id sits at id + odelta + v * osv
    long osv;          // (odelta = 0, osv = G.sv: out has the layout of the other arrays)
};

template <typename T>
__device__ __forceinline__ T fget(const UpdArgs<T> &a, int d, int comp, const int (&p)[3])
{
    return a.ff[d][comp * a.fb[d].sc + a.fb[d].idx(p[0], p[1], p[2])];
}

// Edge EMF E_c at face index fp on axis p=(c+1)%3, face index fq on axis
// q=(c+2)%3 and cell cc on axis c.  Face slot 4 of the p-sweep is B_q, slot 5
// of the q-sweep is B_p.
template <typename T>
__device__ __forceinline__ T emf(const UpdArgs<T> &a, int c, int fp, int fq, int cc)
{
    const int p = (c + 1) % 3, q = (c + 2) % 3;
    const bool ap = a.G.act[p], aq = a.G.act[q];
    int pos[3];
    pos[c] = cc;
    if (ap && aq) {
        pos[p] = fp; pos[q] = fq - 1;
        T t = -fget(a, p, 4, pos);
        pos[q] = fq;
        t -= fget(a, p, 4, pos);
        pos[p] = fp - 1;
        t += fget(a, q, 5, pos);
        pos[p] = fp;
        t += fget(a, q, 5, pos);
        return T(0.25) * t;
    }
    if (ap) { pos[p] = fp; pos[q] = 0; return -fget(a, p, 4, pos); }
    if (aq) { pos[q] = fq; pos[p] = 0; return fget(a, q, 5, pos); }
    return T(0);
}

// d b_n / dt on the n-face fn at transverse cells j1 (axis n+1), j2 (axis n+2).
template <typename T>
__device__ __forceinline__ T face_bdot(const UpdArgs<T> &a, int n, int fn, int j1, int j2)
{
    const int a1 = (n + 1) % 3, a2 = (n + 2) % 3;
    T r = T(0);
    if (a.G.act[a1])
        r -= (emf(a, a2, fn, j1 + 1, j2) - emf(a, a2, fn, j1, j2)) * T(a.G.idl[a1]);
    if (a.G.act[a2])
        r += (emf(a, a1, j2 + 1, fn, j1) - emf(a, a1, j2, fn, j1)) * T(a.G.idl[a2]);
    return r;
}

// RK combination of the variables vars[] of one cell: L[v] is the
// right-hand side of variable v, id the cell's state index; out points at
// the cell's first output variable (variables osv apart).
template <typename T, int NV>
__device__ __forceinline__ void rk_store_vars(const StageCoef &c, long sv, long id, const T *__restrict__ u0,
                                              const T *acc_in, T *acc_out, T *out, long osv,
                                              const int (&vars)[NV], const T (&L)[8])
{
    if (c.mode == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) out[vars[m] * osv] = L[vars[m]];
        return;
    }
    const T bdt = T(c.bdt), cdt = T(c.cdt);
    if (c.mode == 2) {
        const T a0 = T(c.a0), a1 = T(c.a1);
        if (c.a1 != 0.0) {
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                const int v = vars[m];
                out[v * osv] = a0 * u0[id + v * sv] + a1 * acc_in[id + v * sv] + cdt * L[v];
            }
        } else {
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                const int v = vars[m];
                out[v * osv] = a0 * u0[id + v * sv] + cdt * L[v];
            }
        }
        return;
    }
    if (c.s == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const int v = vars[m];
            T w = u0[id + v * sv];
            acc_out[id + v * sv] = w + bdt * L[v];
            out[v * osv] = w + cdt * L[v];
        }
    } else if (c.s < 3) {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const int v = vars[m];
            T w = u0[id + v * sv];
            T ac = acc_in[id + v * sv];
            acc_out[id + v * sv] = ac + bdt * L[v];
            out[v * osv] = w + cdt * L[v];
        }
    } else {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const int v = vars[m];
            out[v * osv] = acc_in[id + v * sv] + cdt * L[v];
        }
    }
}

constexpr int ALL_VARS[8] = { 0, 1, 2, 3, 4, 5, 6, 7 };
constexpr int B_VARS[3] = { 4, 5, 6 };
constexpr int HYDRO_VARS[5] = { 0, 1, 2, 3, 7 };

// RK combination of one cell (all variables, or B only when the hydro part
// of the stage was done by the fused x sweep).
template <typename T>
__device__ __forceinline__ void rk_store(const UpdArgs<T> &a, long id, const T (&L)[8])
{
    T *const out = a.out + (id + a.odelta);
    if (a.c.bonly) rk_store_vars<T, 3>(a.c, a.G.sv, id, a.u0, a.acc_in, a.acc_out, out, a.osv, B_VARS, L);
    else rk_store_vars<T, 8>(a.c, a.G.sv, id, a.u0, a.acc_in, a.acc_out, out, a.osv, ALL_VARS, L);
}

// L(U) of one interior cell at pos (any active axes), then the RK store.
template <typename T>
__device__ __forceinline__ void update_cell(const UpdArgs<T> &a, const int (&pos)[3])
{
    const Geom &G = a.G;
    const long id = G.base + pos[0] * G.s[0] + pos[1] * G.s[1] + (long)pos[2] * G.s[2];
    T L[8] = { T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0) };
    // rho, m, E: flux differences (face slots 0..3 and 6 -> variables 0..3, 7)
    const int hs[5] = { 0, 1, 2, 3, 6 }, hv[5] = { 0, 1, 2, 3, 7 };
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        if (a.c.bonly) break;
        T acc = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (!G.act[d]) continue;
            int pp[3] = { pos[0], pos[1], pos[2] };
            pp[d] = pos[d] + 1;
            T fr = fget(a, d, hs[h], pp);
            pp[d] = pos[d];
            T fl = fget(a, d, hs[h], pp);
            acc -= (fr - fl) * T(G.idl[d]);
        }
        L[hv[h]] = acc;
    }
    // B: constrained transport
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        const int a1 = (n + 1) % 3, a2 = (n + 2) % 3;
        T val;
        if (G.act[n] && a.c.stag)
            val = face_bdot(a, n, pos[n], pos[a1], pos[a2]);     // the lower face itself
        else if (G.act[n])
            val = T(0.5) * (face_bdot(a, n, pos[n], pos[a1], pos[a2])
                            + face_bdot(a, n, pos[n] + 1, pos[a1], pos[a2]));
        else
            val = face_bdot(a, n, 0, pos[a1], pos[a2]);
        L[4 + n] = val;
    }
    rk_store(a, id, L);
}

// Three active axes: the update of cells (i, j, k0..k1-1) of one column,
// marching in k.  The z-face fluxes and the EMFs of the upper z-level are
// carried to the next cell; the EMF of every edge is formed exactly as in
// emf() (same operands, same order), so results equal update_cell's.
// BONLY: only B (CT), the hydro variables having been updated by the fused x
// sweep; the hydro face components are then neither read nor stored.
template <typename T, bool BONLY = false, bool STAG = false>
__device__ __forceinline__ void march_column(const UpdArgs<T> &a, int i, int j, int k0, int k1)
{
    const Geom &G = a.G;
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
    T fzlo[5] = { T(0), T(0), T(0), T(0), T(0) };
    if (!BONLY) {
#pragma unroll
        for (int h = 0; h < 5; ++h) fzlo[h] = FZ[hs[h] * sz + BZ.idx(i, j, k0)];
    }

    for (int k = k0; k < k1; ++k) {
        const long id = G.base + i * G.s[0] + j * G.s[1] + (long)k * G.s[2];
        T L[8] = { T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0) };
        T fzhi[5];
#pragma unroll
        for (int h = 0; h < 5; ++h) {
            if (BONLY) break;
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
        if (STAG) {
            // staggered storage: each B slot is its cell's lower face
            L[4] = bxl;
            L[5] = byl;
            L[6] = bzl;
            (void)bxr; (void)byr; (void)bzr;
        } else {
            L[4] = T(0.5) * (bxl + bxr);
            L[5] = T(0.5) * (byl + byr);
            L[6] = T(0.5) * (bzl + bzr);
        }
        T *const out = a.out + (id + a.odelta);
        if (BONLY) rk_store_vars<T, 3>(a.c, G.sv, id, a.u0, a.acc_in, a.acc_out, out, a.osv, B_VARS, L);
        else rk_store_vars<T, 8>(a.c, G.sv, id, a.u0, a.acc_in, a.acc_out, out, a.osv, ALL_VARS, L);
        // carry to level k+1
        Ey0 = Ey2; Ey1 = Ey3; Ex0 = Ex2; Ex1 = Ex3;
        x5c0 = x5h0; x5c1 = x5h1; y4c0 = y4h0; y4c1 = y4h1;
        if (!BONLY) {
#pragma unroll
            for (int h = 0; h < 5; ++h) fzlo[h] = fzhi[h];
        }
    }
}

// march_column<T, true, false> (B only, cell-centred B) with the loads of
// level k+1 issued before the arithmetic of level k, so that a thread keeps
// one level's loads in flight while it computes: for kernels with few waves
// per SIMD (the batched stage), where the plain march waits a full memory
// latency per level.  Same operands, expressions and order as march_column.
template <typename T>
struct BLevel {
    T x5h0, x5h1, y4h0, y4h1;          // FX5(i|i+1, j, k+1), FY4(i, j|j+1, k+1)
    T z4m, z4c, z4p;                   // FZ4(i-1|i|i+1, j, k+1)
    T z5m, z5c, z5p;                   // FZ5(i, j-1|j|j+1, k+1)
    T x4[6];                           // FX4 at (i, j-1), (i, j), (i+1, j-1), (i+1, j), (i, j+1), (i+1, j+1), level k
    T y5[6];                           // FY5 at (i-1, j), (i, j), (i+1, j), (i-1, j+1), (i, j+1), (i+1, j+1), level k
    T w0[3], w1[3];                    // u0 and acc_in of B at the cell
};

template <typename T>
__device__ __forceinline__ void blevel_load(const UpdArgs<T> &a, int i, int j, int k, bool u0, bool ac,
                                            BLevel<T> &L)
{
    const T *FX = a.ff[0], *FY = a.ff[1], *FZ = a.ff[2];
    const FaceBox &BX = a.fb[0], &BY = a.fb[1], &BZ = a.fb[2];
    const long sx = BX.sc, sy = BY.sc, sz = BZ.sc;
    L.x5h0 = FX[5 * sx + BX.idx(i, j, k + 1)];
    L.x5h1 = FX[5 * sx + BX.idx(i + 1, j, k + 1)];
    L.y4h0 = FY[4 * sy + BY.idx(i, j, k + 1)];
    L.y4h1 = FY[4 * sy + BY.idx(i, j + 1, k + 1)];
    L.z4m = FZ[4 * sz + BZ.idx(i - 1, j, k + 1)];
    L.z4c = FZ[4 * sz + BZ.idx(i, j, k + 1)];
    L.z4p = FZ[4 * sz + BZ.idx(i + 1, j, k + 1)];
    L.z5m = FZ[5 * sz + BZ.idx(i, j - 1, k + 1)];
    L.z5c = FZ[5 * sz + BZ.idx(i, j, k + 1)];
    L.z5p = FZ[5 * sz + BZ.idx(i, j + 1, k + 1)];
    L.x4[0] = FX[4 * sx + BX.idx(i, j - 1, k)];
    L.x4[1] = FX[4 * sx + BX.idx(i, j, k)];
    L.x4[2] = FX[4 * sx + BX.idx(i + 1, j - 1, k)];
    L.x4[3] = FX[4 * sx + BX.idx(i + 1, j, k)];
    L.x4[4] = FX[4 * sx + BX.idx(i, j + 1, k)];
    L.x4[5] = FX[4 * sx + BX.idx(i + 1, j + 1, k)];
    L.y5[0] = FY[5 * sy + BY.idx(i - 1, j, k)];
    L.y5[1] = FY[5 * sy + BY.idx(i, j, k)];
    L.y5[2] = FY[5 * sy + BY.idx(i + 1, j, k)];
    L.y5[3] = FY[5 * sy + BY.idx(i - 1, j + 1, k)];
    L.y5[4] = FY[5 * sy + BY.idx(i, j + 1, k)];
    L.y5[5] = FY[5 * sy + BY.idx(i + 1, j + 1, k)];
    const Geom &G = a.G;
    const long id = G.base + i * G.s[0] + j * G.s[1] + (long)k * G.s[2];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        L.w0[m] = u0 ? a.u0[id + B_VARS[m] * G.sv] : T(0);
        L.w1[m] = ac ? a.acc_in[id + B_VARS[m] * G.sv] : T(0);
    }
}

template <typename T>
__device__ __forceinline__ void march_column_b_pipelined(const UpdArgs<T> &a, int i, int j, int k0, int k1)
{
    const Geom &G = a.G;
    const T *FX = a.ff[0], *FY = a.ff[1], *FZ = a.ff[2];
    const FaceBox &BX = a.fb[0], &BY = a.fb[1], &BZ = a.fb[2];
    const long sx = BX.sc, sy = BY.sc, sz = BZ.sc;
    const T idx = T(G.idl[0]), idy = T(G.idl[1]), idz = T(G.idl[2]);
    const T q = T(0.25);
    const StageCoef &c = a.c;
    const bool u0 = (c.mode == 1 && c.s < 3) || c.mode == 2;
    const bool ac = (c.mode == 1 && c.s > 0) || (c.mode == 2 && c.a1 != 0.0);
    const T bdt = T(c.bdt), cdt = T(c.cdt), a0 = T(c.a0), a1 = T(c.a1);

    // carried values at the lower z-level k0 (as march_column)
    T x5c0 = FX[5 * sx + BX.idx(i, j, k0)], x5c1 = FX[5 * sx + BX.idx(i + 1, j, k0)];
    T y4c0 = FY[4 * sy + BY.idx(i, j, k0)], y4c1 = FY[4 * sy + BY.idx(i, j + 1, k0)];
    T Ey0, Ey1, Ex0, Ex1;
    {
        const T x5lo0 = FX[5 * sx + BX.idx(i, j, k0 - 1)], x5lo1 = FX[5 * sx + BX.idx(i + 1, j, k0 - 1)];
        const T y4lo0 = FY[4 * sy + BY.idx(i, j, k0 - 1)], y4lo1 = FY[4 * sy + BY.idx(i, j + 1, k0 - 1)];
        T t = -FZ[4 * sz + BZ.idx(i - 1, j, k0)];
        t -= FZ[4 * sz + BZ.idx(i, j, k0)];
        t += x5lo0;
        t += x5c0;
        Ey0 = q * t;
        t = -FZ[4 * sz + BZ.idx(i, j, k0)];
        t -= FZ[4 * sz + BZ.idx(i + 1, j, k0)];
        t += x5lo1;
        t += x5c1;
        Ey1 = q * t;
        t = -y4lo0;
        t -= y4c0;
        t += FZ[5 * sz + BZ.idx(i, j - 1, k0)];
        t += FZ[5 * sz + BZ.idx(i, j, k0)];
        Ex0 = q * t;
        t = -y4lo1;
        t -= y4c1;
        t += FZ[5 * sz + BZ.idx(i, j, k0)];
        t += FZ[5 * sz + BZ.idx(i, j + 1, k0)];
        Ex1 = q * t;
    }
    BLevel<T> cur, nxt;
    blevel_load<T>(a, i, j, k0, u0, ac, cur);
    for (int k = k0; k < k1; ++k) {
        if (k + 1 < k1) blevel_load<T>(a, i, j, k + 1, u0, ac, nxt);
        T t;
        t = -cur.z4m; t -= cur.z4c; t += x5c0; t += cur.x5h0; const T Ey2 = q * t;
        t = -cur.z4c; t -= cur.z4p; t += x5c1; t += cur.x5h1; const T Ey3 = q * t;
        t = -y4c0; t -= cur.y4h0; t += cur.z5m; t += cur.z5c; const T Ex2 = q * t;
        t = -y4c1; t -= cur.y4h1; t += cur.z5c; t += cur.z5p; const T Ex3 = q * t;
        t = -cur.x4[0]; t -= cur.x4[1]; t += cur.y5[0]; t += cur.y5[1]; const T Ez00 = q * t;
        t = -cur.x4[2]; t -= cur.x4[3]; t += cur.y5[1]; t += cur.y5[2]; const T Ez10 = q * t;
        t = -cur.x4[1]; t -= cur.x4[4]; t += cur.y5[3]; t += cur.y5[4]; const T Ez01 = q * t;
        t = -cur.x4[3]; t -= cur.x4[5]; t += cur.y5[4]; t += cur.y5[5]; const T Ez11 = q * t;
        T r, bxl, bxr, byl, byr, bzl, bzr;
        r = T(0); r -= (Ez01 - Ez00) * idy; r += (Ey2 - Ey0) * idz; bxl = r;
        r = T(0); r -= (Ez11 - Ez10) * idy; r += (Ey3 - Ey1) * idz; bxr = r;
        r = T(0); r -= (Ex2 - Ex0) * idz; r += (Ez10 - Ez00) * idx; byl = r;
        r = T(0); r -= (Ex3 - Ex1) * idz; r += (Ez11 - Ez01) * idx; byr = r;
        r = T(0); r -= (Ey1 - Ey0) * idx; r += (Ex1 - Ex0) * idy; bzl = r;
        r = T(0); r -= (Ey3 - Ey2) * idx; r += (Ex3 - Ex2) * idy; bzr = r;
        const T Lb[3] = { T(0.5) * (bxl + bxr), T(0.5) * (byl + byr), T(0.5) * (bzl + bzr) };
        const long id = G.base + i * G.s[0] + j * G.s[1] + (long)k * G.s[2];
        T *const out = a.out + (id + a.odelta);
        // rk_store_vars's expressions on the preloaded u0 / acc_in values
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const long o = id + B_VARS[m] * G.sv;
            const long oo = B_VARS[m] * a.osv;
            if (c.mode == 0) {
                out[oo] = Lb[m];
            } else if (c.mode == 2) {
                out[oo] = c.a1 != 0.0 ? a0 * cur.w0[m] + a1 * cur.w1[m] + cdt * Lb[m] : a0 * cur.w0[m] + cdt * Lb[m];
            } else if (c.s == 0) {
                a.acc_out[o] = cur.w0[m] + bdt * Lb[m];
                out[oo] = cur.w0[m] + cdt * Lb[m];
            } else if (c.s < 3) {
                a.acc_out[o] = cur.w1[m] + bdt * Lb[m];
                out[oo] = cur.w0[m] + cdt * Lb[m];
            } else {
                out[oo] = cur.w1[m] + cdt * Lb[m];
            }
        }
        Ey0 = Ey2; Ey1 = Ey3; Ex0 = Ex2; Ex1 = Ex3;
        x5c0 = cur.x5h0; x5c1 = cur.x5h1; y4c0 = cur.y4h0; y4c1 = cur.y4h1;
        if (k + 1 < k1) cur = nxt;
    }
}

}  // namespace up
}  // namespace ww
