// ww_sweep_dev.h -- device code of the characteristic WENO5 sweep, shared by
// the single-box kernels and the batched persistent kernel.
//
// One thread computes the flux at one interface i+1/2 of the sweep axis
// (arXiv:1808.10633, Sec. 2.1, eq. 1 per characteristic field).  A block
// first stages the cells of its tile (plus the 3-cell halo on each side of
// the sweep axis) in LDS together with the per-cell quantities every
// interface needs (pressure, 1/rho, fast/slow/Alfven speeds), so each cell's
// equation of state and wave speeds are evaluated once per block.
//
// Per interface:
//   1. the six stencil cells i-2..i+3 are read from LDS; their physical
//      fluxes are formed; the central combination (-F_{i-1} + 7F_i + 7F_{i+1}
//      - F_{i+2})/12 (kept doubled) and the five cell-to-cell differences of F
//      and U are taken (eq. 1 is linear in these; the projection rows carry the
//      1/2 of the Lax-Friedrichs split, a power-of-two scaling), and the
//      largest |lambda^s| per field over the stencil gives the local
//      Lax-Friedrichs speed;
//   2. the mean state of cells i and i+1 (arithmetic mean of the primitive
//      variables) gives the seven-wave eigen-system with the Roe-Balsara
//      normalisation; the left eigenvectors are applied as
//      L_U X = L_W (dW/dU) X: the Jacobian dW/dU once per vector, then the
//      sparse primitive rows, after rotating the transverse components onto
//      the (B_t, perpendicular) basis, in which every row has at most four
//      entries and the +- members of a wave pair share their terms;
//   3. per field: split F^{s+-} differences, WENO5 weights (eqs. 3-7, with the
//      three weights put over one common denominator), phi_N (eq. 2), eq. (1);
//   4. back-projection R_U F^s = (dU/dW) R_W F^s, again through the sparse
//      primitive columns; the flux is stored in grid components.
// The sweep axis is a template parameter: no data is transposed.
#pragma once
#include "ww_internal.h"
#include "ww_update_dev.h"

#include <math.h>

namespace ww {
namespace sw {

constexpr int NQ = 13;      // staged quantities per cell
// LDS slots: 0 rho, 1 mn, 2 mt1, 3 mt2, 4 Bn, 5 Bt1, 6 Bt2, 7 E,
//            8 p, 9 1/rho, 10 c_f, 11 c_s, 12 c_A   (sweep frame)
// Tiles staged with the cell fluxes (PRE: the FP32 x sweeps) add 13 v_n and
// 14..19 the sweep-frame flux components 1..6 (the mass flux is m_n): every
// cell serves six interfaces, and its flux is then formed once per tile
// instead of once per interface, for 20 quantities of LDS.
constexpr int NQ_PRE = 20;
template <bool PRE> constexpr int nq() { return PRE ? NQ_PRE : NQ; }
constexpr int TILE = 64;    // lanes per row
constexpr int ROWS = 4;     // waves per block
constexpr int NCX = TILE + 5;

// Reciprocal: hardware estimate refined by Newton steps (two in FP64, one in
// FP32), to within rounding of the correctly rounded quotient.
__device__ __forceinline__ double frcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float frcp(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}
// Reciprocal of the nonlinear weights' common denominator.  FP64: one Newton
// step on the estimate, which is good to about 2^-23, leaving a relative error
// near 2^-46 in the weights (about 1e-14), far below the scheme's truncation
// error and the weights' own sensitivity to rounding in the smoothness
// indicators.  FP32: the estimate itself (within 1 ulp).
__device__ __forceinline__ double frcp_w(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float frcp_w(float x) { return __builtin_amdgcn_rcpf(x); }

// Square root in FP64 for finite x >= 0: the hardware reciprocal-square-root
// estimate, one Goldschmidt step towards g = sqrt(x), h = 1/(2 sqrt(x)), then
// a Newton correction g += (x - g^2) h with the residual formed by a fused
// multiply-add (Markstein's formulation).  With exactly rounded FMAs the
// result is the correctly rounded root for estimate errors up to 2^-22 and
// within 1 ulp up to 2^-14.  The estimate is taken at x + 2^-1022, so x = 0
// gives 0 and x < 0 gives NaN; the wave speeds and normalisations passed here
// are never subnormal or infinite, so the range scaling and special-case
// selects of the general routine are left out.
__device__ __forceinline__ double fsqrt(double x)
{
    const double y = __builtin_amdgcn_rsq(x + 0x1p-1022);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}
__device__ __forceinline__ float fsqrt(float x) { return sqrtf(x); }

// 1/sqrt(x) in FP64 for finite x > 0: the estimate refined by two Newton
// steps y += y (1 - x y^2) / 2.
__device__ __forceinline__ double frsq(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
}

// Staging runs at a raised wave priority.  Two blocks share a CU, so while
// one block stages its tile (global loads, equation of state, LDS writes) the
// other is usually deep in its interface arithmetic; without the raise the
// older waves of that block win the issue arbitration and the staging block's
// loads and barrier are delayed.  The raise ends after the staging barrier.
constexpr int STAGE_PRIO = 2;
__device__ __forceinline__ void stage_begin() { __builtin_amdgcn_s_setprio(STAGE_PRIO); }
__device__ __forceinline__ void stage_end() { __builtin_amdgcn_s_setprio(0); }

// Square roots of the scales 18 and 12 that fold the linear weights
// d = (1, 6, 3)/10 and the 1/3, 1/6 of eq. (2) into the (epsilon + IS_k).
constexpr double SQ18 = 4.2426406871192851464, SQ12 = 3.4641016151377545870;

// phi_N of eq. (2) with the weights of eqs. (3)-(7).  ee = (epsilon/4,
// sqrt(18) epsilon/4, sqrt(12) epsilon/4).
// WZ: the WENO-Z weights of Borges et al. (2008) instead (exponent 1, an
// ablation): alpha_k = d_k (1 + tau5 / (eps + IS_k)), tau5 = |IS_0 - IS_2|.
// LBL: also the largest deviation of a weight from the linear weights.
// FOLD: the folded form below (fewer instructions; two more values live).
template <typename T, bool LBL = false, bool WZ = false, bool FOLD = true>
__device__ __forceinline__ T phi_n(T a, T b, T c, T d, const T (&ee)[3], T *dev = nullptr)
{
    if constexpr (!WZ && !LBL && FOLD) {
        // With r_0 = sqrt(18) q_0, r_1 = q_1, r_2 = sqrt(12) q_2 (q_k as
        // below) and R_k = r_k^2: A = R_1 R_2, B = R_0 R_1, C = R_0 R_2 are
        // 12, 6 and 36 times the common-denominator numerators of alpha_0,
        // alpha_2, alpha_1, so omega_0 = 3A / S and omega_2 = 6B / S with
        // S = 3A + 6B + C, and eq. (2) becomes
        //   phi = (A (a-2b+c) + B (b-2c+d)) / S - (b-2c+d)/12
        // (one reciprocal, no separate scaling of the differences).
        const T b2 = b * b, c2 = c * c;
        T r0 = fma(a, fma(T(4 * SQ18), a, T(-11 * SQ18) * b), fma(T(10 * SQ18), b2, ee[1]));
        T r1 = fma(T(4), b2 + c2, fma(T(-5), b * c, ee[0]));
        T r2 = fma(d, fma(T(4 * SQ12), d, T(-11 * SQ12) * c), fma(T(10 * SQ12), c2, ee[2]));
        if constexpr (sizeof(T) == 4) {
            // FP32: keep the products of the squares in range (see below)
            const T s = __builtin_amdgcn_rcpf(fmax(r0, fmax(r1, r2)));
            r0 *= s; r1 *= s; r2 *= s;
        }
        r0 *= r0; r1 *= r1; r2 *= r2;
        const T A = r1 * r2, B = r0 * r1;
        const T inv = frcp_w(fma(T(3), A, fma(T(6), B, r0 * r2)));
        const T y = fma(T(-2), c, b) + d;
        return fma(fma(A, fma(T(-2), b, a) + c, B * y), inv, T(-1.0 / 12.0) * y);
    }
    const T e4 = ee[0];
    // Smoothness indicators of eqs. (5)-(7), expanded into the quadratic forms
    // IS_0 = 16a^2 - 44ab + 40b^2, IS_1 = 16b^2 - 20bc + 16c^2,
    // IS_2 = 40c^2 - 44cd + 16d^2 (all positive definite), and divided by 4
    // together with epsilon: the weights depend only on ratios of the
    // (epsilon + IS_k), so they are unchanged (an exact power-of-two scale).
    T b2 = b * b, c2 = c * c;
    T q0 = fma(a, fma(T(4), a, T(-11) * b), fma(T(10), b2, e4));
    T q1 = fma(T(4), b2 + c2, fma(T(-5), b * c, e4));
    T q2 = fma(d, fma(T(4), d, T(-11) * c), fma(T(10), c2, e4));
    if constexpr (sizeof(T) == 4) {
        // FP32: the products of four (epsilon + IS)/4 below overflow once IS
        // passes ~5e9 (strong blasts); scaled by (about) their largest they
        // stay in (0, 1], and the weights, which depend only on ratios, are
        // unchanged, so the hardware reciprocal estimate serves as the scale
        const T s = __builtin_amdgcn_rcpf(fmax(q0, fmax(q1, q2)));
        q0 *= s; q1 *= s; q2 *= s;
    }
    T n0, n1, n2;
    if constexpr (WZ) {
        // alpha_k = d_k (q_k + t) / q_k with t = |q_0 - q_2| (= tau5 / 4),
        // over the common denominator q0 q1 q2
        const T t = fabs(q0 - q2);
        n0 = (q0 + t) * q1 * q2;
        n1 = T(6) * (q1 + t) * q0 * q2;
        n2 = T(3) * (q2 + t) * q0 * q1;
    } else {
        q0 *= q0; q1 *= q1; q2 *= q2;
        // alpha_k = d_k / q_k with d = (1, 6, 3); omega_k = alpha_k / sum alpha,
        // written over the common denominator q0 q1 q2 (one reciprocal).
        n0 = q1 * q2; n1 = T(6) * q0 * q2; n2 = T(3) * q0 * q1;
    }
    T inv = frcp(n0 + n1 + n2);
    if constexpr (LBL) {
        // largest deviation of (omega_0, omega_1, omega_2) from (0.1, 0.6, 0.3)
        T w0 = n0 * inv, w1 = n1 * inv, w2 = n2 * inv;
        T dv = fmax(fmax(fabs(w0 - T(0.1)), fabs(w1 - T(0.6))), fabs(w2 - T(0.3)));
        *dev = fmax(*dev, dv);
    }
    // eq. (2): omega_0 (a-2b+c)/3 + (omega_2 - 1/2)(b-2c+d)/6
    T x3 = (a - T(2) * b + c) * T(1.0 / 3.0);
    T y6 = (b - T(2) * c + d) * T(1.0 / 6.0);
    return fma(inv, fma(n0, x3, n2 * y6), T(-0.5) * y6);
}

// eq. (1) for one field.  cc: projected central term; df, du: projected flux
// and state differences (k = 0..4 at i-3/2 .. i+5/2), both already carrying
// the 1/2 of the Lax-Friedrichs split; al: LF speed.
template <typename T, bool LBL = false, bool WZ = false, bool FOLD = true>
__device__ __forceinline__ T weno_field(T cc, const T (&df)[5], const T (&du)[5], T al, const T (&ee)[3],
                                        T *dev = nullptr)
{
    T dp[5], dm[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        dp[k] = fma(al, du[k], df[k]);
        dm[k] = fma(-al, du[k], df[k]);
    }
    return cc - phi_n<T, LBL, WZ, FOLD>(dp[0], dp[1], dp[2], dp[3], ee, dev)
              + phi_n<T, LBL, WZ, FOLD>(dm[4], dm[3], dm[2], dm[1], ee, dev);
}

// Sweep-frame physical flux of one cell (rho, mn, mt1, mt2, Bt1, Bt2, E
// components) from its conserved variables w, pressure p and 1/rho; returns
// the normal velocity.
template <typename T>
__device__ __forceinline__ T cell_flux(const T (&w)[8], T p, T ir, T (&F)[7])
{
    const T mn = w[1], m1 = w[2], m2 = w[3], bn = w[4], b1 = w[5], b2 = w[6], e = w[7];
    const T vn = mn * ir, v1 = m1 * ir, v2 = m2 * ir;
    const T pt = p + T(0.5) * (bn * bn + b1 * b1 + b2 * b2);
    F[0] = mn;
    F[1] = mn * vn + pt - bn * bn;
    F[2] = m1 * vn - bn * b1;
    F[3] = m2 * vn - bn * b2;
    F[4] = vn * b1 - v1 * bn;
    F[5] = vn * b2 - v2 * bn;
    F[6] = (e + pt) * vn - bn * (vn * bn + v1 * b1 + v2 * b2);
    return vn;
}

// Stage one cell from its sweep-frame conserved variables w (rho, mn, mt1,
// mt2, Bn, Bt1, Bt2, E): the variables and the derived quantities.  LIN:
// slots 0..10 only (the learned router's routed sweeps: linear fluxes and
// features need no c_s, c_A).
template <typename T, bool PRE = false, bool LIN = false>
__device__ __forceinline__ void stage_values(const T (&w)[8], double gamma, T *q, int qs)
{
    const T r = w[0], mn = w[1], m1 = w[2], m2 = w[3], bn = w[4], b1 = w[5], b2 = w[6], e = w[7];
    // pressure recovery (kept in FP64 for every storage type)
    double ird = frcp((double)r);
    double pd = (gamma - 1.0) * ((double)e - 0.5 * ((double)mn * mn + (double)m1 * m1 + (double)m2 * m2) * ird
                                 - 0.5 * ((double)bn * bn + (double)b1 * b1 + (double)b2 * b2));
    T p = (T)pd;
    T ir = (T)ird;
    T a2 = T(gamma) * p * ir;
    T bn2 = bn * bn * ir;
    T bt2 = (b1 * b1 + b2 * b2) * ir;
    T dd = a2 - bn2;
    T disc = dd * dd + bt2 * (T(2) * a2 + T(2) * bn2 + bt2);
    T cf2 = T(0.5) * (a2 + bn2 + bt2 + fsqrt(disc));
    T cs2 = a2 * bn2 * frcp(cf2);       // (unused, and not computed, with LIN)
    q[0 * qs] = r;  q[1 * qs] = mn; q[2 * qs] = m1; q[3 * qs] = m2;
    q[4 * qs] = bn; q[5 * qs] = b1; q[6 * qs] = b2; q[7 * qs] = e;
    q[8 * qs] = p;
    q[9 * qs] = ir;
    q[10 * qs] = fsqrt(cf2);
    if constexpr (!LIN) {
        q[11 * qs] = fsqrt(cs2);
        q[12 * qs] = fsqrt(bn2);
    }
    if constexpr (PRE) {
        T F[7];
        const T vn = cell_flux(w, p, ir, F);
        q[13 * qs] = vn;
#pragma unroll
        for (int c = 1; c < 7; ++c) q[(13 + c) * qs] = F[c];
    }
}

// Stage one cell: its variables read from the state (cm: sweep-frame order).
template <typename T, bool PRE = false, bool LIN = false>
__device__ __forceinline__ void stage_cell(const T *__restrict__ u, long id, long sv,
                                           const int (&cm)[8], double gamma, T *q, int qs)
{
    T w[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) w[v] = u[id + cm[v] * sv];
    stage_values<T, PRE, LIN>(w, gamma, q, qs);
}

// Stage cells c = tid, tid + 256, ... (< ncell, at most IT per thread) of a
// tile: every global load of the thread's cells first, then the equation of
// state and LDS stores of each.  A thread's loads are then in flight
// together rather than one cell's latency after another's, which matters at
// two waves per SIMD.  cell_id(c, id) gives the state index of tile cell c,
// false if the cell is not staged; c's LDS slot is sq + c.
template <int IT, bool PRE = false, bool LIN = false, typename T, typename CellId>
__device__ __forceinline__ void stage_tile(const T *__restrict__ u, long sv, const int (&cm)[8], double gamma,
                                           T *sq, int qs, int ncell, CellId cell_id)
{
    const int tid = threadIdx.x + TILE * threadIdx.y;
    T w[IT][8];
    bool ok[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int c = tid + it * TILE * ROWS;
        long id = 0;
        ok[it] = c < ncell && cell_id(c, id);
        if (ok[it]) {
#pragma unroll
            for (int v = 0; v < 8; ++v) w[it][v] = u[id + cm[v] * sv];
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it)
        if (ok[it]) stage_values<T, PRE, LIN>(w[it], gamma, sq + tid + it * TILE * ROWS, qs);
}

// Interface flux from six staged cells.  sq: LDS base, qs: stride between
// quantities, off: offset of cell i-2, cstr: stride between cells.
// out: sweep-frame flux (rho, mn, mt1, mt2, Bt1, Bt2, E).
// LBL: also return in *dev the largest deviation of any weight of any field
// from the linear weights (the label of a troubled interface).
// GLF: the LF speed of field s is ag[s] (global speeds of the sweep, an
// ablation) instead of the largest |lambda^s| over the six cells.
// FOLD: phi_n's folded form (off where the register budget is exhausted).
// PRE: the cells were staged with their fluxes and v_n (NQ_PRE quantities).
template <typename T, bool LBL = false, bool WZ = false, bool GLF = false, bool FOLD = true, bool PRE = false>
__device__ __forceinline__ void face_flux(const T *__restrict__ sq, int qs, int off, int cstr,
                                          double gamma, double igm1, T eps, T (&out)[7],
                                          T *dev = nullptr, const double *ag = nullptr)
{
#define QQ(q, j) sq[(q) * qs + off + (j) * cstr]
    T C[7], dY[5][7], dZ[5][7], am[7];
    T Fp[7], Up[7];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        T vn, cf, cs, ca, Fj[7], Uj[7];
        if constexpr (PRE) {
            const T r = QQ(0, j), mn = QQ(1, j), m1 = QQ(2, j), m2 = QQ(3, j);
            const T b1 = QQ(5, j), b2 = QQ(6, j), e = QQ(7, j);
            vn = QQ(13, j); cf = QQ(10, j); cs = QQ(11, j); ca = QQ(12, j);
            Fj[0] = mn;
#pragma unroll
            for (int c = 1; c < 7; ++c) Fj[c] = QQ(13 + c, j);
            Uj[0] = r; Uj[1] = mn; Uj[2] = m1; Uj[3] = m2; Uj[4] = b1; Uj[5] = b2; Uj[6] = e;
        } else {
            // cell_flux's expressions, written out and in this order (the FP64
            // kernels' register allocation at 256 VGPRs follows the order of
            // the LDS reads)
            T r = QQ(0, j), mn = QQ(1, j), m1 = QQ(2, j), m2 = QQ(3, j);
            T bn = QQ(4, j), b1 = QQ(5, j), b2 = QQ(6, j), e = QQ(7, j);
            T p = QQ(8, j), ir = QQ(9, j);
            cf = QQ(10, j); cs = QQ(11, j); ca = QQ(12, j);
            vn = mn * ir;
            T v1 = m1 * ir, v2 = m2 * ir;
            T pt = p + T(0.5) * (bn * bn + b1 * b1 + b2 * b2);
            Fj[0] = mn; Fj[1] = mn * vn + pt - bn * bn; Fj[2] = m1 * vn - bn * b1; Fj[3] = m2 * vn - bn * b2;
            Fj[4] = vn * b1 - v1 * bn; Fj[5] = vn * b2 - v2 * bn;
            Fj[6] = (e + pt) * vn - bn * (vn * bn + v1 * b1 + v2 * b2);
            Uj[0] = r; Uj[1] = mn; Uj[2] = m1; Uj[3] = m2; Uj[4] = b1; Uj[5] = b2; Uj[6] = e;
        }
        T lam[7] = { fabs(vn - cf), fabs(vn - ca), fabs(vn - cs), fabs(vn),
                     fabs(vn + cs), fabs(vn + ca), fabs(vn + cf) };
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            am[c] = (j == 0) ? lam[c] : fmax(am[c], lam[c]);
            if (j == 1) C[c] = -Fj[c];
            if (j == 2 || j == 3) C[c] += T(7) * Fj[c];
            if (j == 4) C[c] = (C[c] - Fj[c]) * T(1.0 / 6.0);   // twice the central term
            if (j > 0) { dY[j - 1][c] = Fj[c] - Fp[c]; dZ[j - 1][c] = Uj[c] - Up[c]; }
            Fp[c] = Fj[c];
            Up[c] = Uj[c];
        }
    }
    if constexpr (GLF) {
#pragma unroll
        for (int c = 0; c < 7; ++c) am[c] = T(ag[c]);
    }

    // Interface state: mean of the primitive variables of cells i and i+1.
    // Eigen-system normalisation in FP64 for every storage type.
    double r2 = QQ(0, 2), r3 = QQ(0, 3), i2 = QQ(9, 2), i3 = QQ(9, 3);
    double rb = 0.5 * (r2 + r3);
    double vnb = 0.5 * ((double)QQ(1, 2) * i2 + (double)QQ(1, 3) * i3);
    double v1b = 0.5 * ((double)QQ(2, 2) * i2 + (double)QQ(2, 3) * i3);
    double v2b = 0.5 * ((double)QQ(3, 2) * i2 + (double)QQ(3, 3) * i3);
    double bnb = 0.5 * ((double)QQ(4, 2) + (double)QQ(4, 3));
    double b1b = 0.5 * ((double)QQ(5, 2) + (double)QQ(5, 3));
    double b2b = 0.5 * ((double)QQ(6, 2) + (double)QQ(6, 3));
    double pb = 0.5 * ((double)QQ(8, 2) + (double)QQ(8, 3));
#undef QQ
    // FP32 storage: 1/rho, a and 1/a^2, c_f and 1/c_f^2 from one reciprocal
    // square root each, and c_s = a c_A / c_f with c_A = |B_n| rho^-1/2.  The
    // FP64 kernels sit at the 256-VGPR limit, where the longer live ranges of
    // that form spill; they take each quantity separately.
    constexpr bool LEAN = sizeof(T) == 4;
    double irb, isr = 0.0;
    if constexpr (LEAN) { isr = frsq(rb); irb = isr * isr; }
    else irb = frcp(rb);
    double a2 = gamma * pb * irb;
    double bn2 = bnb * bnb * irb;
    double bt2 = (b1b * b1b + b2b * b2b) * irb;
    double dd = a2 - bn2;
    double sqD = fsqrt(dd * dd + bt2 * (2.0 * a2 + 2.0 * bn2 + bt2));
    double cf2 = 0.5 * (a2 + bn2 + bt2 + sqD);
    double icf2, rcf = 0.0, cs2 = 0.0;
    if constexpr (LEAN) { rcf = frsq(cf2); icf2 = rcf * rcf; }
    else { icf2 = frcp(cf2); cs2 = a2 * bn2 * icf2; }
    double af, as;
    if (sqD <= 1e-12 * (a2 + bn2 + bt2)) {
        af = 1.0; as = 0.0;
    } else {
        // (cf^2 - a^2)(cf^2 - bn^2) = bt^2 cf^2 avoids the cancellation
        double P, Q;
        if (dd >= 0.0) { P = 0.5 * (dd + bt2 + sqD); Q = bt2 * cf2 * frcp(P); }
        else           { Q = 0.5 * (-dd + bt2 + sqD); P = bt2 * cf2 * frcp(Q); }
        double isq = frcp(sqD);
        double af2 = fmin(fmax(a2 * P * icf2 * isq, 0.0), 1.0);
        double as2 = fmin(fmax(Q * isq, 0.0), 1.0);
        af = fsqrt(af2); as = fsqrt(as2);
    }
    double be1, be2;
    if (bt2 > 1e-24 * (a2 + bn2)) {
        double ibt = frsq(b1b * b1b + b2b * b2b);
        be1 = b1b * ibt; be2 = b2b * ibt;
    } else {
        // B_t ~ 0: any unit vector spans the degenerate wave pairs; the first
        // transverse axis keeps the two transverse momenta in separate
        // characteristic fields, so a planar flow (no component or gradient
        // along one transverse axis) stays planar
        be1 = 1.0; be2 = 0.0;
    }
    double sg = (bnb >= 0.0) ? 1.0 : -1.0;
    double cfm, csm, am_, ia2;
    if constexpr (LEAN) {
        const double ra = frsq(a2);
        am_ = a2 * ra; ia2 = ra * ra;
        cfm = cf2 * rcf; csm = am_ * fabs(bnb) * isr * rcf;
    } else {
        cfm = fsqrt(cf2); csm = fsqrt(cs2); am_ = fsqrt(a2);
        isr = frsq(rb); ia2 = frcp(a2);
    }
    const double sr = rb * isr;
    double gm1 = gamma - 1.0;
    double hv2 = 0.5 * (vnb * vnb + v1b * v1b + v2b * v2b);

    // rows of L_W, per wave pair: odd (sign-flipping) and even parts, with
    // the 1/2 of the Lax-Friedrichs split folded in (exact power-of-two scale)
    // and the 1/rho and (gamma - 1) of dW/dU: xf below leaves the velocity
    // components rho times and the pressure 1/(gamma - 1) times too large, and
    // every row entry that multiplies them carries the inverse factor
    const double i2a2 = 0.25 * ia2, ir2 = i2a2 * irb, ig2 = i2a2 * gm1 * irb;
    const T kf1 = T(af * cfm * ir2), kf2 = T(as * csm * sg * ir2);
    const T kf4 = T(as * am_ * isr * i2a2), kf6 = T(af * ig2);
    const T ks1 = T(as * csm * ir2), ks2 = T(af * cfm * sg * ir2);
    const T ks4 = T(af * am_ * isr * i2a2), ks6 = T(as * ig2);
    const T ka3 = T(0.25 * sg * irb), ka5 = T(0.25 * isr), ke6 = T(ia2 * gm1), kh = T(0.5);

    // dW/dU at the interface state (without the two scales above) followed by
    // the rotation of the transverse components onto (beta, perpendicular).
    const T tv = T(vnb), t1 = T(v1b), t2 = T(v2b), th = T(hv2);
    const T tb1 = T(b1b), tb2 = T(b2b), e1 = T(be1), e2 = T(be2);
    auto xf = [&](T (&X)[7]) {
        T w1 = X[1] - tv * X[0];
        T w2 = X[2] - t1 * X[0];
        T w3 = X[3] - t2 * X[0];
        T w6 = th * X[0] - tv * X[1] - t1 * X[2] - t2 * X[3] - tb1 * X[4] - tb2 * X[5] + X[6];
        T pv = e1 * w2 + e2 * w3, qv = e2 * w2 - e1 * w3;
        T pB = e1 * X[4] + e2 * X[5], qB = e1 * X[5] - e2 * X[4];
        X[1] = w1; X[2] = pv; X[3] = qv; X[4] = pB; X[5] = qB; X[6] = w6;
    };
    xf(C);
#pragma unroll
    for (int k = 0; k < 5; ++k) { xf(dY[k]); xf(dZ[k]); }

    T G[7] = { T(0), T(0), T(0), T(0), T(0), T(0), T(0) };
    const T teps = T(0.25) * eps;     // epsilon / 4 for phi_n
    const T ee[3] = { teps, teps * T(SQ18), teps * T(SQ12) };

    // One wave pair (sigma = -1 field index lo, sigma = +1 field index hi).
    // proj(X, odd, even) gives the odd and even parts of the row applied to X.
    auto pair = [&](auto proj, int lo, int hi, T &S, T &D) {
        T oc, ec, odf[5], edf[5], odu[5], edu[5];
        proj(C, oc, ec);
#pragma unroll
        for (int k = 0; k < 5; ++k) { proj(dY[k], odf[k], edf[k]); proj(dZ[k], odu[k], edu[k]); }
        T df[5], du[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) { df[k] = edf[k] + odf[k]; du[k] = edu[k] + odu[k]; }
        T fplus = weno_field<T, LBL, WZ, FOLD>(ec + oc, df, du, am[hi], ee, dev);
#pragma unroll
        for (int k = 0; k < 5; ++k) { df[k] = edf[k] - odf[k]; du[k] = edu[k] - odu[k]; }
        T fminus = weno_field<T, LBL, WZ, FOLD>(ec - oc, df, du, am[lo], ee, dev);
        S = fplus + fminus;
        D = fplus - fminus;
    };

    T S, D;
    // fast pair (fields 0 and 6)
    pair([&](const T (&X)[7], T &o, T &e) { o = kf1 * X[1] - kf2 * X[2]; e = kf4 * X[4] + kf6 * X[6]; },
         0, 6, S, D);
    {
        const T c0 = T(rb * af), c1 = T(af * cfm), c2 = T(-as * csm * sg), c4 = T(as * sr * am_),
                c6 = T(rb * af * a2);
        G[0] += c0 * S; G[1] += c1 * D; G[2] += c2 * D; G[4] += c4 * S; G[6] += c6 * S;
    }
    // slow pair (fields 2 and 4)
    pair([&](const T (&X)[7], T &o, T &e) { o = ks1 * X[1] + ks2 * X[2]; e = ks6 * X[6] - ks4 * X[4]; },
         2, 4, S, D);
    {
        const T c0 = T(rb * as), c1 = T(as * csm), c2 = T(af * cfm * sg), c4 = T(-af * sr * am_),
                c6 = T(rb * as * a2);
        G[0] += c0 * S; G[1] += c1 * D; G[2] += c2 * D; G[4] += c4 * S; G[6] += c6 * S;
    }
    // Alfven pair (fields 1 and 5)
    pair([&](const T (&X)[7], T &o, T &e) { o = ka3 * X[3]; e = ka5 * X[5]; }, 1, 5, S, D);
    G[3] += T(sg) * D;
    G[5] += T(sr) * S;
    // entropy (field 3)
    {
        T cc = kh * (C[0] - ke6 * C[6]), df[5], du[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            df[k] = kh * (dY[k][0] - ke6 * dY[k][6]);
            du[k] = kh * (dZ[k][0] - ke6 * dZ[k][6]);
        }
        G[0] += weno_field<T, LBL, WZ, FOLD>(cc, df, du, am[3], ee, dev);
    }

    // back to (vt1, vt2), (Bt1, Bt2) and through dU/dW
    T gv1 = e1 * G[2] + e2 * G[3], gv2 = e2 * G[2] - e1 * G[3];
    T gb1 = e1 * G[4] - e2 * G[5], gb2 = e2 * G[4] + e1 * G[5];
    const T trb = T(rb);
    out[0] = G[0];
    out[1] = tv * G[0] + trb * G[1];
    out[2] = t1 * G[0] + trb * gv1;
    out[3] = t2 * G[0] + trb * gv2;
    out[4] = gb1;
    out[5] = gb2;
    out[6] = th * G[0] + trb * (tv * G[1] + t1 * gv1 + t2 * gv2) + tb1 * gb1 + tb2 * gb2
           + G[6] * T(igm1);
}

// Linear fifth-order component-wise flux of the six staged cells (the cheap
// flux of interfaces the learned router calls smooth): one Lax-Friedrichs
// speed alpha = max(|v_n| + c_f) over the stencil for every component and
// the linear-weight form of eq. (1), (2,-13,47,27,-3)/60 on F^+ and the
// mirror (-3,27,47,-13,2)/60 on F^-.  With F^+- = (F +- alpha U)/2 the two
// stencils add up to the sixth-order central combination of F,
// (1,-8,37,37,-8,1)/60, plus alpha times the fifth difference of U,
// (1,-5,10,-10,5,-1)/60: the same flux in 12 operations per component.
template <typename T>
__device__ __forceinline__ void linear_flux(const T *__restrict__ sq, int qs, int off, int cstr,
                                            T (&out)[7])
{
#define QL(q, j) sq[(q) * qs + off + (j) * cstr]
    T F[6][7], U[6][7], al = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        T r = QL(0, j), mn = QL(1, j), m1 = QL(2, j), m2 = QL(3, j);
        T bn = QL(4, j), b1 = QL(5, j), b2 = QL(6, j), e = QL(7, j);
        T p = QL(8, j), ir = QL(9, j), cf = QL(10, j);
        T vn = mn * ir, v1 = m1 * ir, v2 = m2 * ir;
        T pt = p + T(0.5) * (bn * bn + b1 * b1 + b2 * b2);
        F[j][0] = mn; F[j][1] = mn * vn + pt - bn * bn; F[j][2] = m1 * vn - bn * b1;
        F[j][3] = m2 * vn - bn * b2; F[j][4] = vn * b1 - v1 * bn; F[j][5] = vn * b2 - v2 * bn;
        F[j][6] = (e + pt) * vn - bn * (vn * bn + v1 * b1 + v2 * b2);
        U[j][0] = r; U[j][1] = mn; U[j][2] = m1; U[j][3] = m2; U[j][4] = b1; U[j][5] = b2; U[j][6] = e;
        al = fmax(al, fabs(vn) + cf);
    }
#undef QL
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        const T cen = fma(T(37), F[2][c] + F[3][c], fma(T(-8), F[1][c] + F[4][c], F[0][c] + F[5][c]));
        const T dis = fma(T(10), U[2][c] - U[3][c], fma(T(-5), U[1][c] - U[4][c], U[0][c] - U[5][c]));
        out[c] = fma(al, dis, cen) * T(1.0 / 60.0);
    }
}

// Store a sweep-frame interface flux in grid components:
// rho, mx, my, mz, B_(N+1), B_(N+2), E.
template <int N, typename T>
__device__ __forceinline__ void store_face(T *__restrict__ flux, const FaceBox &F, const int (&pos)[3],
                                           const T (&out)[7])
{
    constexpr int T1 = (N + 1) % 3, T2 = (N + 2) % 3;
    const long fi = F.idx(pos[0], pos[1], pos[2]);
    flux[0 * F.sc + fi] = out[0];
    flux[(1 + N) * F.sc + fi] = out[1];
    flux[(1 + T1) * F.sc + fi] = out[2];
    flux[(1 + T2) * F.sc + fi] = out[3];
    flux[4 * F.sc + fi] = out[4];
    flux[5 * F.sc + fi] = out[5];
    flux[6 * F.sc + fi] = out[6];
}

// Periodic image of cell index x (-n <= x < 2n) in 0..n-1.  WRAP tiles (the
// batched form's periodic patches) stage each ghost cell from its image
// directly, so the patch needs no ghost fill.
__device__ __forceinline__ int pwrap(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

template <int DIR, int FT>
__host__ __device__ constexpr int tile_cells() { return DIR == 0 ? ROWS * NCX : TILE * (FT + 5); }

// One tile of interfaces along axis DIR.  x sweep: ROWS rows (transverse
// (j,k) pairs, tile index ta) x TILE consecutive faces (tile index tb).
// y/z sweeps: TILE consecutive positions of the transverse plane (x fastest,
// tile index ta) x FT consecutive faces (tile index tb); each of the ROWS
// waves computes faces w, w+ROWS, ...  sq: LDS of NQ * tile_cells<DIR,FT>()
// elements.  Ends with a block barrier, so consecutive tiles may reuse sq.
// LF: stage with stage_tile (a thread's loads first: the batched kernel, at
// two waves per SIMD, gains 4 %; the single-box FP32 y/z sweeps lose 1 %).
template <int DIR, int FT, typename T, bool WZ = false, bool GLF = false, bool WRAP = false, bool LF = false>
__device__ __forceinline__ void sweep_tile(const T *__restrict__ u, T *__restrict__ flux,
                                           const Geom &G, const FaceBox &F, const Phys &P,
                                           int ta, int tb, T *sq)
{
    constexpr int N = DIR, T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
    const int cm[8] = { 0, 1 + N, 1 + T1, 1 + T2, 4 + N, 4 + T1, 4 + T2, 7 };
    constexpr int NC = tile_cells<DIR, FT>();
    const int lane = threadIdx.x, w = threadIdx.y, tid = lane + TILE * w;
    const int nlast = G.n[N] + 2;   // last cell index along the sweep axis

    stage_begin();
    if constexpr (DIR == 0) {
        const int nrows = F.cnt[1] * F.cnt[2];
        const int r0 = ta * ROWS;
        const int f0 = tb * TILE;
        auto cell_id = [&](int c, long &id) {
            const int rr = c / NCX, xi = c - rr * NCX;
            const int row = r0 + rr;
            int x = f0 - 3 + xi;
            if (row >= nrows || x > nlast) return false;
            int j = F.lo[1] + row % F.cnt[1], k = F.lo[2] + row / F.cnt[1];
            if (WRAP) { x = pwrap(x, G.n[0]); j = pwrap(j, G.n[1]); k = pwrap(k, G.n[2]); }
            id = G.base + x * G.s[0] + j * G.s[1] + k * G.s[2];
            return true;
        };
        if constexpr (LF) {
            stage_tile<(ROWS * NCX + 255) / 256>(u, G.sv, cm, P.gamma, sq, NC, ROWS * NCX, cell_id);
        } else {
            for (int c = tid; c < ROWS * NCX; c += TILE * ROWS) {
                long id;
                if (cell_id(c, id)) stage_cell(u, id, G.sv, cm, P.gamma, sq + c, NC);
            }
        }
        __syncthreads();
        stage_end();
        const int row = r0 + w;
        int pos[3];
        pos[0] = f0 + lane;
        pos[1] = F.lo[1] + row % F.cnt[1];
        pos[2] = F.lo[2] + row / F.cnt[1];
        if (row < nrows && pos[0] < F.cnt[0]) {
            T out[7];
            face_flux<T, false, WZ, GLF>(sq, NC, w * NCX + lane, 1, P.gamma, P.igm1, (T)P.eps, out, nullptr,
                                         P.ag);
            store_face<N, T>(flux, F, pos, out);
        }
    } else {
        // positions in the transverse plane (x fastest, then the other axis)
        constexpr int A = 0, B = (DIR == 1) ? 2 : 1;
        const int npos = F.cnt[A] * F.cnt[B];
        const int p = ta * TILE + lane;
        const int f0 = tb * FT;
        const int ca = F.lo[A] + p % F.cnt[A], cb = F.lo[B] + p / F.cnt[A];
        const int wa = WRAP ? pwrap(ca, G.n[A]) : ca, wb = WRAP ? pwrap(cb, G.n[B]) : cb;
        // cell c = rr * TILE + lane: row rr of the tile at this thread's position
        auto cell_id = [&](int c, long &id) {
            int y = f0 - 3 + c / TILE;
            if (p >= npos || y > nlast) return false;
            if (WRAP) y = pwrap(y, G.n[N]);
            id = G.base + wa * G.s[A] + wb * G.s[B] + (long)y * G.s[N];
            return true;
        };
        if constexpr (LF) {
            stage_tile<(NC + 255) / 256>(u, G.sv, cm, P.gamma, sq, NC, NC, cell_id);
        } else {
            for (int c = tid; c < NC; c += TILE * ROWS) {
                long id;
                if (cell_id(c, id)) stage_cell(u, id, G.sv, cm, P.gamma, sq + c, NC);
            }
        }
        __syncthreads();
        stage_end();
        for (int ff = w; ff < FT; ff += ROWS) {
            int pos[3];
            pos[A] = ca;
            pos[B] = cb;
            pos[N] = f0 + ff;
            if (p < npos && pos[N] < F.cnt[N]) {
                T out[7];
                face_flux<T, false, WZ, GLF>(sq, NC, ff * TILE + lane, TILE, P.gamma, P.igm1, (T)P.eps, out,
                                             nullptr, P.ag);
                store_face<N, T>(flux, F, pos, out);
            }
        }
    }
    __syncthreads();
}

// The rho, m, E update of one cell in the fused x sweeps, in two parts:
// fused_cell_load issues the cell's global loads (its y and z faces' fluxes
// and the RK arrays the stage form reads) before the tile's barrier, so that
// they are in flight while the other waves finish their face fluxes;
// fused_cell_rk forms L from the two x faces' fluxes and the loaded values
// (the update kernel's expressions and order: x, y, z) and stores the RK
// combination (rk_store_vars's expressions: identical results);
// fused_cell_store takes the x fluxes from LDS.
template <typename T>
struct FusedCell {
    T fyl[5], fyr[5], fzl[5], fzr[5], w0[5], w1[5];
    long id;
};

template <typename T>
__device__ __forceinline__ void fused_cell_load(const XFuse<T> &xf, const Geom &G, int i, int j, int k,
                                                FusedCell<T> &c)
{
    const int hs[5] = { 0, 1, 2, 3, 6 }, hv[5] = { 0, 1, 2, 3, 7 };
    c.id = G.base + i * G.s[0] + j * G.s[1] + (long)k * G.s[2];
    const long yl = xf.by.idx(i, j, k), yr = xf.by.idx(i, j + 1, k);
    const long zl = xf.bz.idx(i, j, k), zr = xf.bz.idx(i, j, k + 1);
    const StageCoef &q = xf.c;
    const bool u0 = (q.mode == 1 && q.s < 3) || q.mode == 2;
    const bool ac = (q.mode == 1 && q.s > 0) || (q.mode == 2 && q.a1 != 0.0);
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        c.fyl[h] = xf.fy[hs[h] * xf.by.sc + yl];
        c.fyr[h] = xf.fy[hs[h] * xf.by.sc + yr];
        c.fzl[h] = xf.fz[hs[h] * xf.bz.sc + zl];
        c.fzr[h] = xf.fz[hs[h] * xf.bz.sc + zr];
        c.w0[h] = u0 ? xf.u0[c.id + hv[h] * G.sv] : T(0);
        c.w1[h] = ac ? xf.acc_in[c.id + hv[h] * G.sv] : T(0);
    }
}

template <typename T>
__device__ __forceinline__ void fused_cell_rk(const XFuse<T> &xf, const Geom &G, const T (&xl)[5], const T (&xr)[5],
                                              const FusedCell<T> &c)
{
    const int hv[5] = { 0, 1, 2, 3, 7 };
    const T idx = T(G.idl[0]), idy = T(G.idl[1]), idz = T(G.idl[2]);
    const StageCoef &q = xf.c;
    const T bdt = T(q.bdt), cdt = T(q.cdt), a0 = T(q.a0), a1 = T(q.a1);
    const long sv = G.sv, id = c.id;
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        T L = T(0);
        L -= (xr[h] - xl[h]) * idx;
        L -= (c.fyr[h] - c.fyl[h]) * idy;
        L -= (c.fzr[h] - c.fzl[h]) * idz;
        const long o = id + hv[h] * sv;
        if (q.mode == 0) {
            xf.out[o] = L;
        } else if (q.mode == 2) {
            xf.out[o] = q.a1 != 0.0 ? a0 * c.w0[h] + a1 * c.w1[h] + cdt * L : a0 * c.w0[h] + cdt * L;
        } else if (q.s == 0) {
            xf.acc_out[o] = c.w0[h] + bdt * L;
            xf.out[o] = c.w0[h] + cdt * L;
        } else if (q.s < 3) {
            xf.acc_out[o] = c.w1[h] + bdt * L;
            xf.out[o] = c.w0[h] + cdt * L;
        } else {
            xf.out[o] = c.w1[h] + cdt * L;
        }
    }
}

// The cell between tile faces tid and tid + 1, whose rho, m, E fluxes are in
// LDS (hx, nh apart per component).
template <typename T>
__device__ __forceinline__ void fused_cell_store(const XFuse<T> &xf, const Geom &G, const T *hx, int nh, int tid,
                                                 const FusedCell<T> &c)
{
    T xl[5], xr[5];
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        xl[h] = hx[h * nh + tid];
        xr[h] = hx[h * nh + tid + 1];
    }
    fused_cell_rk<T>(xf, G, xl, xr, c);
}

// x sweep for short rows (batched patches): the block takes XF_FACES
// consecutive faces of the flattened (row, face) space, stages every cell of
// the rows they touch (-3..n+2), and each thread computes XF_FPT faces (one:
// two faces per thread spill registers at two waves per SIMD, and the
// batched FP32 step measured 4% slower).  The rows touched hold at most
// xflat_cells(n, rows) cells; sq needs NQ * XF_MAXC elements.  Face and row
// numbers are 32-bit: a patch (edges of at most 1024 cells) has at most
// 1025 * 1026^2 < 2^31 x faces, and 64-bit divisions are long software
// sequences on the GPU.
constexpr int XF_FPT = 1;
constexpr int XF_FACES = TILE * ROWS * XF_FPT;
constexpr int XF_MAXC = 544;     // 4-cell rows: at most 53 rows of 10 cells
__host__ __device__ inline int xflat_cells(int nx, long nrows)
{
    long span = (XF_FACES + nx) / (nx + 1) + 1;
    if (span > nrows) span = nrows;
    return (int)(span * (nx + 6));
}

// Stage every cell of the rows that faces g0 .. g0+XF_FACES-1 touch; returns
// the first row (sq with stride XF_MAXC).
template <typename T, bool WRAP = false>
__device__ __forceinline__ long xflat_stage(const T *__restrict__ u, const Geom &G, const FaceBox &F, const Phys &P,
                                            long g0, T *sq)
{
    const int cm[8] = { 0, 1, 2, 3, 4, 5, 6, 7 };
    const int nf = F.cnt[0], rowc = G.n[0] + 6;
    const int nrows = F.cnt[1] * F.cnt[2];
    const int r_lo = (int)g0 / nf;
    int r_hi = ((int)g0 + XF_FACES - 1) / nf;
    if (r_hi > nrows - 1) r_hi = nrows - 1;
    const int ncell = (r_hi - r_lo + 1) * rowc;
    stage_tile<(XF_MAXC + 255) / 256>(u, G.sv, cm, P.gamma, sq, XF_MAXC, ncell, [&](int c, long &id) {
        const int row = r_lo + c / rowc;
        int x = c % rowc - 3;
        int j = F.lo[1] + row % F.cnt[1], k = F.lo[2] + row / F.cnt[1];
        if (WRAP) { x = pwrap(x, G.n[0]); j = pwrap(j, G.n[1]); k = pwrap(k, G.n[2]); }
        id = G.base + x * G.s[0] + j * G.s[1] + k * G.s[2];
        return true;
    });
    return r_lo;
}

// The flattened x sweep with the rho, m, E part of the update fused in (the
// batched form's counterpart of sweep_tile_xseg_fused): tiles of XF_FACES
// faces overlapping by one (tile t starts at face (XF_FACES-1) t), the
// fluxes' rho, m, E in LDS (hx, 5 x XF_FACES); thread tid takes faces
// tid + q TILE ROWS (q < XF_FPT) and the cell right of each when the next
// face is in the same row and the row is interior: x, y, z differences in
// the update kernel's order and expressions, then the RK combination.  Only
// the transverse-B fluxes of the x faces are stored.  Ends with a block
// barrier.
template <typename T, bool WRAP = false>
__device__ __forceinline__ void sweep_tile_xflat_fused(const T *__restrict__ u, T *__restrict__ flux,
                                                       const Geom &G, const FaceBox &F, const Phys &P,
                                                       long tile, T *sq, T *hx, const XFuse<T> &xf)
{
    constexpr int NT = TILE * ROWS, STRIDE = XF_FACES - 1;
    const int nf = F.cnt[0], rowc = G.n[0] + 6;
    const int total = F.cnt[1] * F.cnt[2] * nf;
    const int g0 = (int)tile * STRIDE;
    const int tid = threadIdx.x + TILE * threadIdx.y;
    stage_begin();
    const int r_lo = (int)xflat_stage<T, WRAP>(u, G, F, P, g0, sq);
    __syncthreads();
    stage_end();
    int pos[XF_FPT][3];
    bool valid[XF_FPT];
#pragma unroll
    for (int q = 0; q < XF_FPT; ++q) {
        const int f = tid + q * NT, g = g0 + f;
        valid[q] = g < total;
        pos[q][0] = pos[q][1] = pos[q][2] = 0;
        if (valid[q]) {
            const int row = g / nf;
            pos[q][0] = g - row * nf;
            pos[q][1] = F.lo[1] + row % F.cnt[1];
            pos[q][2] = F.lo[2] + row / F.cnt[1];
            T out[7];
            face_flux<T>(sq, XF_MAXC, (row - r_lo) * rowc + pos[q][0], 1, P.gamma, P.igm1, (T)P.eps, out);
            hx[0 * XF_FACES + f] = out[0];
            hx[1 * XF_FACES + f] = out[1];
            hx[2 * XF_FACES + f] = out[2];
            hx[3 * XF_FACES + f] = out[3];
            hx[4 * XF_FACES + f] = out[6];
            if (f < STRIDE || g == total - 1) {
                const long fi = F.idx(pos[q][0], pos[q][1], pos[q][2]);
                flux[4 * F.sc + fi] = out[4];
                flux[5 * F.sc + fi] = out[5];
            }
        }
    }
    // both cells' global loads in flight before the barrier
    FusedCell<T> fc[XF_FPT];
    bool cell[XF_FPT];
#pragma unroll
    for (int q = 0; q < XF_FPT; ++q) {
        const int f = tid + q * NT, g = g0 + f;
        const int i = pos[q][0], j = pos[q][1], k = pos[q][2];
        cell[q] = valid[q] && f < STRIDE && g + 1 < total && i + 1 < nf && j >= 0 && j < G.n[1] && k >= 0 &&
                  k < G.n[2];
        if (cell[q]) fused_cell_load<T>(xf, G, i, j, k, fc[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < XF_FPT; ++q)
        if (cell[q]) fused_cell_store<T>(xf, G, hx, XF_FACES, tid + q * NT, fc[q]);
    __syncthreads();
}

// x sweep over the flattened (row, face) space, for rows of at least
// XSEG_MIN faces: tile t takes the TILE*ROWS consecutive faces t*256 ..
// of the row-major face sequence, which touch at most 4 rows; for each row
// it stages the cells of its face segment with the 3 + 2 halo (256 + 5*4
// cells at most, the size of the regular x tile) and each thread takes one
// face.  Only the last tile of the sweep is ragged.
constexpr int XSEG_MIN = 86;
constexpr int XSEG_CELLS = ROWS * NCX;

// Segment table of one tile: segment s = faces fa_s.. of row r_lo + s at
// transverse cell (j_s, k_s), staged from LDS offset o_s, holding tile-local
// faces from b_s on.  Kept in scalars (a dynamically indexed array would
// live in scratch), and the row -> (j, k) divisions are done once per
// segment, not per cell.
struct XSeg {
    long g0;
    int nf, nface, fa0, fa1, fa2, fa3, o1, o2, o3, o4, b1, b2, b3;
    int j0, j1, j2, j3, k0, k1, k2, k3;
    __device__ int fa(int s) const { return s == 0 ? fa0 : s == 1 ? fa1 : s == 2 ? fa2 : fa3; }
    __device__ int off(int s) const { return s == 0 ? 0 : s == 1 ? o1 : s == 2 ? o2 : o3; }
    __device__ int bs(int s) const { return s == 0 ? 0 : s == 1 ? b1 : s == 2 ? b2 : b3; }
    __device__ int j(int s) const { return s == 0 ? j0 : s == 1 ? j1 : s == 2 ? j2 : j3; }
    __device__ int k(int s) const { return s == 0 ? k0 : s == 1 ? k1 : s == 2 ? k2 : k3; }
};

// stride: first face of tile t is t * stride (TILE*ROWS, or TILE*ROWS - 1 for
// tiles that overlap by one face).
__device__ __forceinline__ XSeg xseg_setup(const FaceBox &F, long tile, int stride = TILE * ROWS)
{
    constexpr int TF = TILE * ROWS;
    XSeg X;
    X.nf = F.cnt[0];
    const long total = (long)F.cnt[1] * F.cnt[2] * X.nf;
    X.g0 = tile * stride;
    const long g1 = (X.g0 + TF - 1 < total - 1) ? X.g0 + TF - 1 : total - 1;
    X.nface = (int)(g1 - X.g0 + 1);
    const long r_lo = X.g0 / X.nf;
    const int nseg = (int)(g1 / X.nf - r_lo) + 1;      // <= 4 since nf >= XSEG_MIN
    X.fa0 = X.fa1 = X.fa2 = X.fa3 = X.o1 = X.o2 = X.o3 = X.o4 = X.b1 = X.b2 = X.b3 = 0;
    X.j0 = X.j1 = X.j2 = X.j3 = X.k0 = X.k1 = X.k2 = X.k3 = 0;
    int o = 0, bsum = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int a = s == 0 ? (int)(X.g0 - r_lo * X.nf) : 0;
        const int b = s == nseg - 1 ? (int)(g1 - (r_lo + s) * X.nf) : X.nf - 1;
        const long row = r_lo + s;
        const int jj = F.lo[1] + (int)(row % F.cnt[1]), kk = F.lo[2] + (int)(row / F.cnt[1]);
        o += s < nseg ? b - a + 6 : 0;
        bsum += s < nseg ? b - a + 1 : 0;                // faces of segments 0..s
        if (s == 0) { X.fa0 = a; X.o1 = o; X.b1 = bsum; X.j0 = jj; X.k0 = kk; }
        if (s == 1) { X.fa1 = a; X.o2 = o; X.b2 = bsum; X.j1 = jj; X.k1 = kk; }
        if (s == 2) { X.fa2 = a; X.o3 = o; X.b3 = bsum; X.j2 = jj; X.k2 = kk; }
        if (s == 3) { X.fa3 = a; X.o4 = o; X.j3 = jj; X.k3 = kk; }
    }
    return X;
}

// Stage the tile's cells (x sweep frame), sq with stride XSEG_CELLS.
template <typename T, bool PRE = false, bool LIN = false>
__device__ __forceinline__ void xseg_stage(const T *__restrict__ u, const Geom &G, const FaceBox & /*F*/,
                                           const Phys &P, const XSeg &X, T *sq)
{
    const int cm[8] = { 0, 1, 2, 3, 4, 5, 6, 7 };
    stage_tile<(XSEG_CELLS + 255) / 256, PRE, LIN>(u, G.sv, cm, P.gamma, sq, XSEG_CELLS, X.o4,
                                                  [&](int c, long &id) {
        const int s = (c >= X.o1) + (c >= X.o2) + (c >= X.o3);
        const int x = X.fa(s) - 3 + (c - X.off(s));
        id = G.base + x * G.s[0] + X.j(s) * G.s[1] + (long)X.k(s) * G.s[2];
        return true;
    });
}

// Face of thread tid: position and LDS offset of its cell i-2 (stride 1).
__device__ __forceinline__ bool xseg_face(const FaceBox & /*F*/, const XSeg &X, int tid, int (&pos)[3], int &off)
{
    const int t = tid < X.nface ? tid : X.nface - 1;
    const int s = (t >= X.b1) + (t >= X.b2) + (t >= X.b3);
    const int f = X.fa(s) + (t - X.bs(s));
    pos[0] = f;
    pos[1] = X.j(s);
    pos[2] = X.k(s);
    off = X.off(s) + (f - X.fa(s));      // stencil cells f-3 .. f+2 from segment offset f - fa
    return tid < X.nface;
}

template <typename T, bool WZ = false, bool GLF = false, bool PRE = false>
__device__ __forceinline__ void sweep_tile_xseg(const T *__restrict__ u, T *__restrict__ flux,
                                                const Geom &G, const FaceBox &F, const Phys &P,
                                                long tile, T *sq)
{
    stage_begin();
    const XSeg X = xseg_setup(F, tile);
    xseg_stage<T, PRE>(u, G, F, P, X, sq);
    __syncthreads();
    stage_end();
    int pos[3], off;
    if (xseg_face(F, X, threadIdx.x + TILE * threadIdx.y, pos, off)) {
        T out[7];
        face_flux<T, false, WZ, GLF, true, PRE>(sq, XSEG_CELLS, off, 1, P.gamma, P.igm1, (T)P.eps, out, nullptr,
                                                P.ag);
        store_face<0, T>(flux, F, pos, out);
    }
}

// The x sweep with the hydro part of the update fused in.  Tiles of 256
// faces overlap by one (tile t starts at face 255 t of the row-major face
// sequence), so both faces of every cell of a row meet in one tile.  After
// the fluxes, each thread puts its face's rho, m, E fluxes in LDS (hx, 5 x
// 256), and thread tid takes the cell between faces tid and tid+1 when both
// lie in one row and the row is interior: its x difference from LDS, its y
// and z differences from the other sweeps' face fluxes (same expressions
// and order as the update kernel: the results are identical), then the RK
// combination of rho, m, E.  Only the transverse-B fluxes (slots 4, 5) are
// stored, once per face (the overlapping face by the next tile).
constexpr int XFUSE_STRIDE = TILE * ROWS - 1;

template <typename T, bool WZ = false, bool GLF = false, bool PRE = false>
__device__ __forceinline__ void sweep_tile_xseg_fused(const T *__restrict__ u, T *__restrict__ flux,
                                                      const Geom &G, const FaceBox &F, const Phys &P,
                                                      long tile, T *sq, T *hx, const XFuse<T> &xf)
{
    stage_begin();
    const XSeg X = xseg_setup(F, tile, XFUSE_STRIDE);
    xseg_stage<T, PRE>(u, G, F, P, X, sq);
    __syncthreads();
    stage_end();
    const int tid = threadIdx.x + TILE * threadIdx.y;
    constexpr int NH = TILE * ROWS;
    int pos[3], off;
    const bool valid = xseg_face(F, X, tid, pos, off);
    if (valid) {
        T out[7];
        face_flux<T, false, WZ, GLF, true, PRE>(sq, XSEG_CELLS, off, 1, P.gamma, P.igm1, (T)P.eps, out, nullptr,
                                                P.ag);
        hx[0 * NH + tid] = out[0];
        hx[1 * NH + tid] = out[1];
        hx[2 * NH + tid] = out[2];
        hx[3 * NH + tid] = out[3];
        hx[4 * NH + tid] = out[6];
        const long total = (long)F.cnt[1] * F.cnt[2] * F.cnt[0];
        if (tid < XFUSE_STRIDE || X.g0 + tid == total - 1) {
            const long fi = F.idx(pos[0], pos[1], pos[2]);
            flux[4 * F.sc + fi] = out[4];
            flux[5 * F.sc + fi] = out[5];
        }
    }
    // the cell between faces tid and tid + 1 of one row (face f sits at f - 1/2)
    const int i = pos[0], j = pos[1], k = pos[2];
    const bool cell = valid && tid < XFUSE_STRIDE && tid + 1 < X.nface && i + 1 < F.cnt[0] && j >= 0 &&
                      j < G.n[1] && k >= 0 && k < G.n[2];
    FusedCell<T> fc;
    if (cell) fused_cell_load<T>(xf, G, i, j, k, fc);
    __syncthreads();
    if (cell) fused_cell_store<T>(xf, G, hx, NH, tid, fc);
}

// y or z sweep with PW positions of the transverse plane (x fastest) per
// tile and 256/PW faces along the sweep, one face per thread: fewer
// positions per tile stage fewer halo cells per face ((FT+5)/FT) in the
// same LDS.
template <int PW>
__host__ __device__ constexpr int yz_cells() { return PW * (256 / PW + 5); }

template <int DIR, int PW, typename T, bool LIN = false>
__device__ __forceinline__ void yz_stage(const T *__restrict__ u, const Geom &G, const FaceBox &F,
                                         const Phys &P, int ta, int tb, T *sq)
{
    constexpr int N = DIR, T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
    constexpr int FTY = 256 / PW, NC = yz_cells<PW>();
    constexpr int A = 0, B = (DIR == 1) ? 2 : 1;
    const int cm[8] = { 0, 1 + N, 1 + T1, 1 + T2, 4 + N, 4 + T1, 4 + T2, 7 };
    const int tid = threadIdx.x + TILE * threadIdx.y;
    const int nlast = G.n[N] + 2;
    const int npos = F.cnt[A] * F.cnt[B];
    const int f0 = tb * FTY;
    // one cell after another (a thread's loads first, as stage_tile does,
    // measured 2 % slower here)
    for (int c = tid; c < NC; c += 256) {
        const int rr = c / PW, pc = c - rr * PW;
        const int p = ta * PW + pc, y = f0 - 3 + rr;
        if (p < npos && y <= nlast) {
            const int ca = F.lo[A] + p % F.cnt[A], cb = F.lo[B] + p / F.cnt[A];
            const long id = G.base + ca * G.s[A] + cb * G.s[B] + (long)y * G.s[N];
            stage_cell<T, false, LIN>(u, id, G.sv, cm, P.gamma, sq + c, NC);
        }
    }
}

// Face of thread tid: position and LDS offset of its cell i-2 (stride PW).
template <int DIR, int PW>
__device__ __forceinline__ bool yz_face(const FaceBox &F, int ta, int tb, int tid, int (&pos)[3], int &off)
{
    constexpr int FTY = 256 / PW, N = DIR, A = 0, B = (DIR == 1) ? 2 : 1;
    const int npos = F.cnt[A] * F.cnt[B];
    const int fr = tid / PW, pl = tid - fr * PW;
    const int p = ta * PW + pl;
    pos[A] = F.lo[A] + p % F.cnt[A];
    pos[B] = F.lo[B] + p / F.cnt[A];
    pos[N] = tb * FTY + fr;
    off = fr * PW + pl;
    return p < npos && pos[N] < F.cnt[N];
}

template <int DIR, int PW, typename T, bool WZ = false, bool GLF = false>
__device__ __forceinline__ void sweep_tile_yz(const T *__restrict__ u, T *__restrict__ flux,
                                              const Geom &G, const FaceBox &F, const Phys &P,
                                              int ta, int tb, T *sq)
{
    stage_begin();
    yz_stage<DIR, PW, T>(u, G, F, P, ta, tb, sq);
    __syncthreads();
    stage_end();
    int pos[3], off;
    if (yz_face<DIR, PW>(F, ta, tb, threadIdx.x + TILE * threadIdx.y, pos, off)) {
        T out[7];
        face_flux<T, false, WZ, GLF>(sq, yz_cells<PW>(), off, PW, P.gamma, P.igm1, (T)P.eps, out, nullptr,
                                     P.ag);
        store_face<DIR, T>(flux, F, pos, out);
    }
}

// Number of tiles (ta, tb) of a sweep.
template <int DIR, int FT>
__host__ __device__ inline void sweep_tiles(const FaceBox &F, long &na, long &nb)
{
    if (DIR == 0) {
        na = ((long)F.cnt[1] * F.cnt[2] + ROWS - 1) / ROWS;
        nb = (F.cnt[0] + TILE - 1) / TILE;
    } else {
        constexpr int B = (DIR == 1) ? 2 : 1;
        na = ((long)F.cnt[0] * F.cnt[B] + TILE - 1) / TILE;
        nb = (F.cnt[DIR] + FT - 1) / FT;
    }
}

}  // namespace sw
}  // namespace ww
