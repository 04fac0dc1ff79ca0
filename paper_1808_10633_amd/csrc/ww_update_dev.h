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
//   Then the low-storage classical RK4 update of the stage.
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

// RK combination of one cell.
template <typename T>
__device__ __forceinline__ void rk_store(const UpdArgs<T> &a, long id, const T (&L)[8])
{
    const StageCoef &c = a.c;
    const long sv = a.G.sv;
    if (c.mode == 0) {
#pragma unroll
        for (int v = 0; v < 8; ++v) a.out[id + v * sv] = L[v];
        return;
    }
    const T bdt = T(c.bdt), cdt = T(c.cdt);
    if (c.s == 0) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            T u0 = a.u0[id + v * sv];
            a.acc_out[id + v * sv] = u0 + bdt * L[v];
            a.out[id + v * sv] = u0 + cdt * L[v];
        }
    } else if (c.s < 3) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            T u0 = a.u0[id + v * sv];
            T ac = a.acc_in[id + v * sv];
            a.acc_out[id + v * sv] = ac + bdt * L[v];
            a.out[id + v * sv] = u0 + cdt * L[v];
        }
    } else {
#pragma unroll
        for (int v = 0; v < 8; ++v) a.out[id + v * sv] = a.acc_in[id + v * sv] + cdt * L[v];
    }
}

// L(U) of one interior cell at pos (any active axes), then the RK store.
template <typename T>
__device__ __forceinline__ void update_cell(const UpdArgs<T> &a, const int (&pos)[3])
{
    const Geom &G = a.G;
    const long id = G.base + pos[0] * G.s[0] + pos[1] * G.s[1] + (long)pos[2] * G.s[2];
    T L[8];
    // rho, m, E: flux differences (face slots 0..3 and 6 -> variables 0..3, 7)
    const int hs[5] = { 0, 1, 2, 3, 6 }, hv[5] = { 0, 1, 2, 3, 7 };
#pragma unroll
    for (int h = 0; h < 5; ++h) {
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
        if (G.act[n])
            val = T(0.5) * (face_bdot(a, n, pos[n], pos[a1], pos[a2])
                            + face_bdot(a, n, pos[n] + 1, pos[a1], pos[a2]));
        else
            val = face_bdot(a, n, 0, pos[a1], pos[a2]);
        L[4 + n] = val;
    }
    rk_store(a, id, L);
}

}  // namespace up
}  // namespace ww
