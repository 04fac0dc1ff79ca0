/*
 * wombat_oracle.c -- serial FP64 CPU oracle for the WENO5 ideal-MHD stage.
 * (Built a second time with OpenMP, the k-plane loops of the sweeps, the
 * flux differences and the RK combinations run on several host threads; each
 * value is computed by the same code either way, so both builds agree bit
 * for bit.)
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  It shares no code
 * with the HIP library.  Plain, slow and written to be checked against the
 * paper by eye: one interface at a time, full 8x8 matrices, no blocking or
 * fusion.
 *
 * Citations are to Donnert et al., arXiv:1808.10633 ("WENO-Wombat"):
 *   Sec. 2.1 eq. (1)      WENO interface flux of one characteristic field
 *   Sec. 2.1 eq. (2)      the WENO5 interpolant phi_N
 *   Sec. 2.1 eqs. (3)-(4) nonlinear weights omega_0, omega_2 and alpha_k
 *   Sec. 2.1 eqs. (5)-(7) smoothness indicators IS_0..IS_2, epsilon = 1e-6
 *   Sec. 2.1              Roe-type decoupling of the 8 PDEs, LF splitting,
 *                         4-stage 4th-order Runge-Kutta, constrained transport
 *                         on a staggered mesh after Ryu et al. (1998)
 *   Sec. 2.2              3 ghost zones, unsplit x/y/z sweeps, final update
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes of the repository):
 *   - the "IC_k" of eq. (4) is the IS_k of eqs. (5)-(7); epsilon is added to
 *     IS unscaled;
 *   - Delta F^{s+-}_{j+1/2} = F^{s+-}_{j+1} - F^{s+-}_j with
 *     F^{s+-} = (L_s.F +- alpha^s L_s.U)/2, all projected with the
 *     interface's left eigenvectors;
 *   - the interface state is the arithmetic mean of the primitive variables
 *     of the two adjacent cells;
 *   - alpha^s is the largest |lambda^s| over the six stencil cells;
 *   - eigenvectors: the seven-wave system at fixed normal field with the
 *     Roe-Balsara normalisation, built in primitive variables and mapped to
 *     conserved ones; the normal-field equation is an identity row with a
 *     zero flux;
 *   - Heaviside-Lorentz units (magnetic pressure B^2/2), ideal-gas EOS;
 *   - CT: edge EMFs are the four-face arithmetic mean of the transverse-B
 *     fluxes; the cell-centred field is advanced by the mean of the two
 *     staggered-face updates;
 *   - classical RK4; dt = C / max sum_d (|v_d| + c_f,d)/dx_d.
 */
#include "wombat_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, BX = 4, BY = 5, BZ = 6, EN = 7 };

/* Degeneracy conventions for the eigenvectors (the paper is silent). */
#define ORC_BT_TINY  1e-24   /* |B_t|^2/rho below this * (a^2 + b_n^2): beta = (1,0) */
#define ORC_CFS_TINY 1e-12   /* c_f^2 - c_s^2 below this * (a^2 + b^2): alpha_f=1, alpha_s=0 */

/* ------------------------------------------------------------------------ */
/* Scalar WENO5, Sec. 2.1 eqs. (2)-(7).                                     */
/* ------------------------------------------------------------------------ */

/* Smoothness indicators (eqs. 5-7) and normalised weights (eqs. 3-4).
 * omega[1] = 1 - omega[0] - omega[2] is returned for the tests. */
void orc_weno_weights(double a, double b, double c, double d, double eps,
                      double omega[3], double is[3])
{
    double is0 = 13.0 * (a - b) * (a - b) + 3.0 * (a - 3.0 * b) * (a - 3.0 * b);
    double is1 = 13.0 * (b - c) * (b - c) + 3.0 * (b + c) * (b + c);
    double is2 = 13.0 * (c - d) * (c - d) + 3.0 * (3.0 * c - d) * (3.0 * c - d);
    double al0 = 1.0 / ((eps + is0) * (eps + is0));
    double al1 = 6.0 / ((eps + is1) * (eps + is1));
    double al2 = 3.0 / ((eps + is2) * (eps + is2));
    double sum = al0 + al1 + al2;
    omega[0] = al0 / sum;
    omega[1] = al1 / sum;
    omega[2] = al2 / sum;
    if (is) { is[0] = is0; is[1] = is1; is[2] = is2; }
}

/* WENO-Z weights (Borges, Carmona, Costa & Don 2008; an ablation, not the
 * paper's scheme, which keeps the weights of eq. 3 and argues in Sec. 2.1
 * that they are the more robust choice): with the same IS_k and
 * tau5 = |IS_0 - IS_2|, alpha_k = d_k (1 + tau5 / (eps + IS_k)), exponent 1. */
void orc_weno_weights_z(double a, double b, double c, double d, double eps,
                        double omega[3], double is[3])
{
    double is0 = 13.0 * (a - b) * (a - b) + 3.0 * (a - 3.0 * b) * (a - 3.0 * b);
    double is1 = 13.0 * (b - c) * (b - c) + 3.0 * (b + c) * (b + c);
    double is2 = 13.0 * (c - d) * (c - d) + 3.0 * (3.0 * c - d) * (3.0 * c - d);
    double tau = fabs(is0 - is2);
    double al0 = 1.0 * (1.0 + tau / (eps + is0));
    double al1 = 6.0 * (1.0 + tau / (eps + is1));
    double al2 = 3.0 * (1.0 + tau / (eps + is2));
    double sum = al0 + al1 + al2;
    omega[0] = al0 / sum;
    omega[1] = al1 / sum;
    omega[2] = al2 / sum;
    if (is) { is[0] = is0; is[1] = is1; is[2] = is2; }
}

static double phi_mode(int z, double a, double b, double c, double d, double eps)
{
    double w[3];
    if (z) orc_weno_weights_z(a, b, c, d, eps, w, NULL);
    else orc_weno_weights(a, b, c, d, eps, w, NULL);
    return w[0] * (a - 2.0 * b + c) / 3.0 + (w[2] - 0.5) * (b - 2.0 * c + d) / 6.0;
}

/* The WENO5 interpolant phi_N(a,b,c,d), eq. (2). */
double orc_weno_phi(double a, double b, double c, double d, double eps)
{
    return phi_mode(0, a, b, c, d, eps);
}

static double field_flux_mode(int z, const double f[6], const double u[6], double alpha,
                              double eps);

/* Interface flux of one decoupled field, eq. (1).
 * f[0..5], u[0..5]: the field's projected flux and state at cells i-2..i+3;
 * the interface is i+1/2.  Lax-Friedrichs splitting with speed alpha. */
double orc_weno_field_flux(const double f[6], const double u[6], double alpha,
                           double eps)
{
    return field_flux_mode(0, f, u, alpha, eps);
}

/* The same with the WENO-Z weights (ablation). */
double orc_weno_field_flux_z(const double f[6], const double u[6], double alpha,
                             double eps)
{
    return field_flux_mode(1, f, u, alpha, eps);
}

static double field_flux_mode(int z, const double f[6], const double u[6], double alpha,
                              double eps)
{
    double fp[6], fm[6], dp[5], dm[5];
    int j;
    for (j = 0; j < 6; ++j) {
        fp[j] = 0.5 * (f[j] + alpha * u[j]);
        fm[j] = 0.5 * (f[j] - alpha * u[j]);
    }
    /* dp[k], dm[k] sit at half index i - 3/2 + k */
    for (j = 0; j < 5; ++j) {
        dp[j] = fp[j + 1] - fp[j];
        dm[j] = fm[j + 1] - fm[j];
    }
    double central = (-f[1] + 7.0 * f[2] + 7.0 * f[3] - f[4]) / 12.0;
    return central
         - phi_mode(z, dp[0], dp[1], dp[2], dp[3], eps)
         + phi_mode(z, dm[4], dm[3], dm[2], dm[1], eps);
}

/* ------------------------------------------------------------------------ */
/* Ideal MHD: EOS, flux, wave speeds (Heaviside-Lorentz units).              */
/* ------------------------------------------------------------------------ */

void orc_prim_to_cons(const double W[8], double gamma, double U[8])
{
    double rho = W[0];
    double v2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
    double b2 = W[4] * W[4] + W[5] * W[5] + W[6] * W[6];
    U[RHO] = rho;
    U[MX] = rho * W[1];
    U[MY] = rho * W[2];
    U[MZ] = rho * W[3];
    U[BX] = W[4];
    U[BY] = W[5];
    U[BZ] = W[6];
    U[EN] = W[7] / (gamma - 1.0) + 0.5 * rho * v2 + 0.5 * b2;
}

void orc_cons_to_prim(const double U[8], double gamma, double W[8])
{
    double rho = U[RHO];
    double vx = U[MX] / rho, vy = U[MY] / rho, vz = U[MZ] / rho;
    double kin = 0.5 * (U[MX] * vx + U[MY] * vy + U[MZ] * vz);
    double mag = 0.5 * (U[BX] * U[BX] + U[BY] * U[BY] + U[BZ] * U[BZ]);
    W[0] = rho;
    W[1] = vx; W[2] = vy; W[3] = vz;
    W[4] = U[BX]; W[5] = U[BY]; W[6] = U[BZ];
    W[7] = (gamma - 1.0) * (U[EN] - kin - mag);
}

/* Flux of the 8 conserved variables along axis dir (0,1,2). */
void orc_flux(const double U[8], int dir, double gamma, double F[8])
{
    double W[8];
    orc_cons_to_prim(U, gamma, W);
    const double *v = W + 1, *B = W + 4;
    double p = W[7];
    double pt = p + 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    double vdotb = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    double vn = v[dir], bn = B[dir];
    int c;
    F[RHO] = U[MX + dir];
    for (c = 0; c < 3; ++c)
        F[MX + c] = U[MX + c] * vn - bn * B[c] + (c == dir ? pt : 0.0);
    for (c = 0; c < 3; ++c)
        F[BX + c] = (c == dir) ? 0.0 : vn * B[c] - v[c] * bn;
    F[EN] = (U[EN] + pt) * vn - bn * vdotb;
}

/* Fast, Alfven and slow speeds along axis dir. */
void orc_wave_speeds(const double U[8], int dir, double gamma,
                     double *cf, double *ca, double *cs)
{
    double W[8];
    orc_cons_to_prim(U, gamma, W);
    double rho = W[0];
    double a2 = gamma * W[7] / rho;
    double bn2 = W[4 + dir] * W[4 + dir] / rho;
    double bt2 = (W[4] * W[4] + W[5] * W[5] + W[6] * W[6]) / rho - bn2;
    if (bt2 < 0.0) bt2 = 0.0;
    double d = a2 - bn2;
    double disc = d * d + bt2 * (2.0 * a2 + 2.0 * bn2 + bt2);
    double cf2 = 0.5 * (a2 + bn2 + bt2 + sqrt(disc));
    double cs2 = a2 * bn2 / cf2;
    *cf = sqrt(cf2);
    *cs = sqrt(cs2);
    *ca = sqrt(bn2);
}

/* ------------------------------------------------------------------------ */
/* Characteristic system (Sec. 2.1: Roe-type decoupling of the 8 PDEs).     */
/* ------------------------------------------------------------------------ */

/* Sweep-frame ordering of the conserved vector:
 *   (rho, mn, mt1, mt2, Bn, Bt1, Bt2, E)
 * and of the seven-wave primitive vector:
 *   (rho, vn, vt1, vt2, Bt1, Bt2, p).
 * Field order: 0 fast-, 1 Alfven-, 2 slow-, 3 entropy, 4 slow+, 5 Alfven+,
 * 6 fast+, 7 the normal-field identity (zero flux). */
static const int m7[7] = { 0, 1, 2, 3, 5, 6, 7 };

static void matmul7(double A[7][7], double B[7][7], double C[7][7])
{
    int r, c, k;
    for (r = 0; r < 7; ++r)
        for (c = 0; c < 7; ++c) {
            double s = 0.0;
            for (k = 0; k < 7; ++k) s += A[r][k] * B[k][c];
            C[r][c] = s;
        }
}

void orc_eigensystem(const double Wn[8], double gamma,
                     double lam[8], double L[64], double R[64])
{
    double rho = Wn[0], vn = Wn[1], vt1 = Wn[2], vt2 = Wn[3];
    double Bn = Wn[4], Bt1 = Wn[5], Bt2 = Wn[6], p = Wn[7];
    double sr = sqrt(rho);
    double a2 = gamma * p / rho, a = sqrt(a2);
    double bn2 = Bn * Bn / rho;
    double bt2 = (Bt1 * Bt1 + Bt2 * Bt2) / rho;
    double d = a2 - bn2;
    double sqD = sqrt(d * d + bt2 * (2.0 * a2 + 2.0 * bn2 + bt2));
    double cf2 = 0.5 * (a2 + bn2 + bt2 + sqD);
    double cs2 = a2 * bn2 / cf2;
    double cf = sqrt(cf2), cs = sqrt(cs2), ca = sqrt(bn2);
    double af, as;
    /* Roe-Balsara normalisation: alpha_f^2 = (a^2-cs^2)/(cf^2-cs^2),
     * alpha_s^2 = (cf^2-a^2)/(cf^2-cs^2), using the identity
     * (cf^2-a^2)(cf^2-bn^2) = bt^2 cf^2 to avoid cancellation. */
    if (sqD <= ORC_CFS_TINY * (a2 + bn2 + bt2)) {
        af = 1.0; as = 0.0;
    } else {
        double P, Q;   /* P = cf^2 - bn^2, Q = cf^2 - a^2 */
        if (d >= 0.0) { P = 0.5 * (d + bt2 + sqD); Q = bt2 * cf2 / P; }
        else          { Q = 0.5 * (-d + bt2 + sqD); P = bt2 * cf2 / Q; }
        double af2 = a2 * P / (cf2 * sqD);
        double as2 = Q / sqD;
        af2 = af2 < 0.0 ? 0.0 : (af2 > 1.0 ? 1.0 : af2);
        as2 = as2 < 0.0 ? 0.0 : (as2 > 1.0 ? 1.0 : as2);
        af = sqrt(af2); as = sqrt(as2);
    }
    double b1, b2;
    if (bt2 > ORC_BT_TINY * (a2 + bn2)) {
        double bt = sqrt(Bt1 * Bt1 + Bt2 * Bt2);
        b1 = Bt1 / bt; b2 = Bt2 / bt;
    } else {
        /* any unit vector spans the degenerate pair; the first transverse
         * axis keeps the two transverse momenta in separate characteristic
         * fields, so a flow without a component or gradient along one
         * transverse axis gains none there */
        b1 = 1.0; b2 = 0.0;
    }
    double s = (Bn >= 0.0) ? 1.0 : -1.0;

    lam[0] = vn - cf; lam[1] = vn - ca; lam[2] = vn - cs; lam[3] = vn;
    lam[4] = vn + cs; lam[5] = vn + ca; lam[6] = vn + cf; lam[7] = 0.0;

    /* Primitive right eigenvectors (columns) and left eigenvectors (rows). */
    double RW[7][7], LW[7][7];
    memset(RW, 0, sizeof RW);
    memset(LW, 0, sizeof LW);
    int k;
    for (k = 0; k < 2; ++k) {
        double sg = (k == 0) ? -1.0 : 1.0;
        int cfast = (k == 0) ? 0 : 6, calf = (k == 0) ? 1 : 5, cslow = (k == 0) ? 2 : 4;
        /* fast */
        RW[0][cfast] = rho * af;
        RW[1][cfast] = sg * af * cf;
        RW[2][cfast] = -sg * as * cs * s * b1;
        RW[3][cfast] = -sg * as * cs * s * b2;
        RW[4][cfast] = as * sr * a * b1;
        RW[5][cfast] = as * sr * a * b2;
        RW[6][cfast] = rho * af * a2;
        LW[cfast][1] = sg * af * cf / (2.0 * a2);
        LW[cfast][2] = -sg * as * cs * s * b1 / (2.0 * a2);
        LW[cfast][3] = -sg * as * cs * s * b2 / (2.0 * a2);
        LW[cfast][4] = as * a * b1 / (sr * 2.0 * a2);
        LW[cfast][5] = as * a * b2 / (sr * 2.0 * a2);
        LW[cfast][6] = af / (rho * 2.0 * a2);
        /* Alfven */
        RW[2][calf] = sg * s * b2;
        RW[3][calf] = -sg * s * b1;
        RW[4][calf] = -sr * b2;
        RW[5][calf] = sr * b1;
        LW[calf][2] = 0.5 * sg * s * b2;
        LW[calf][3] = -0.5 * sg * s * b1;
        LW[calf][4] = -0.5 * b2 / sr;
        LW[calf][5] = 0.5 * b1 / sr;
        /* slow */
        RW[0][cslow] = rho * as;
        RW[1][cslow] = sg * as * cs;
        RW[2][cslow] = sg * af * cf * s * b1;
        RW[3][cslow] = sg * af * cf * s * b2;
        RW[4][cslow] = -af * sr * a * b1;
        RW[5][cslow] = -af * sr * a * b2;
        RW[6][cslow] = rho * as * a2;
        LW[cslow][1] = sg * as * cs / (2.0 * a2);
        LW[cslow][2] = sg * af * cf * s * b1 / (2.0 * a2);
        LW[cslow][3] = sg * af * cf * s * b2 / (2.0 * a2);
        LW[cslow][4] = -af * a * b1 / (sr * 2.0 * a2);
        LW[cslow][5] = -af * a * b2 / (sr * 2.0 * a2);
        LW[cslow][6] = as / (rho * 2.0 * a2);
    }
    /* entropy */
    RW[0][3] = 1.0;
    LW[3][0] = 1.0;
    LW[3][6] = -1.0 / a2;

    /* Jacobians of the map between primitive and conserved variables. */
    double v2 = vn * vn + vt1 * vt1 + vt2 * vt2, gm1 = gamma - 1.0;
    double dUdW[7][7], dWdU[7][7];
    memset(dUdW, 0, sizeof dUdW);
    memset(dWdU, 0, sizeof dWdU);
    dUdW[0][0] = 1.0;
    dUdW[1][0] = vn;  dUdW[1][1] = rho;
    dUdW[2][0] = vt1; dUdW[2][2] = rho;
    dUdW[3][0] = vt2; dUdW[3][3] = rho;
    dUdW[4][4] = 1.0;
    dUdW[5][5] = 1.0;
    dUdW[6][0] = 0.5 * v2; dUdW[6][1] = rho * vn; dUdW[6][2] = rho * vt1;
    dUdW[6][3] = rho * vt2; dUdW[6][4] = Bt1; dUdW[6][5] = Bt2;
    dUdW[6][6] = 1.0 / gm1;
    dWdU[0][0] = 1.0;
    dWdU[1][0] = -vn / rho;  dWdU[1][1] = 1.0 / rho;
    dWdU[2][0] = -vt1 / rho; dWdU[2][2] = 1.0 / rho;
    dWdU[3][0] = -vt2 / rho; dWdU[3][3] = 1.0 / rho;
    dWdU[4][4] = 1.0;
    dWdU[5][5] = 1.0;
    dWdU[6][0] = 0.5 * gm1 * v2; dWdU[6][1] = -gm1 * vn; dWdU[6][2] = -gm1 * vt1;
    dWdU[6][3] = -gm1 * vt2; dWdU[6][4] = -gm1 * Bt1; dWdU[6][5] = -gm1 * Bt2;
    dWdU[6][6] = gm1;

    double RU[7][7], LU[7][7];
    matmul7(dUdW, RW, RU);
    matmul7(LW, dWdU, LU);

    int r, c;
    for (r = 0; r < 64; ++r) { L[r] = 0.0; R[r] = 0.0; }
    for (r = 0; r < 7; ++r)
        for (c = 0; c < 7; ++c) {
            R[m7[r] * 8 + c] = RU[r][c];
            L[r * 8 + m7[c]] = LU[r][c];
        }
    R[4 * 8 + 7] = 1.0;
    L[7 * 8 + 4] = 1.0;
}

/* Largest deviation of the nonlinear weights of eq. (3) from the linear
 * weights (0.1, 0.6, 0.3) for the two phi_N of eq. (1) of one field. */
static double weight_deviation(const double f[6], const double u[6], double alpha,
                               double eps)
{
    double fp[6], fm[6], dp[5], dm[5], w[3], dev = 0.0;
    static const double d[3] = { 0.1, 0.6, 0.3 };
    int j, k;
    for (j = 0; j < 6; ++j) {
        fp[j] = 0.5 * (f[j] + alpha * u[j]);
        fm[j] = 0.5 * (f[j] - alpha * u[j]);
    }
    for (j = 0; j < 5; ++j) { dp[j] = fp[j + 1] - fp[j]; dm[j] = fm[j + 1] - fm[j]; }
    orc_weno_weights(dp[0], dp[1], dp[2], dp[3], eps, w, NULL);
    for (k = 0; k < 3; ++k) if (fabs(w[k] - d[k]) > dev) dev = fabs(w[k] - d[k]);
    orc_weno_weights(dm[4], dm[3], dm[2], dm[1], eps, w, NULL);
    for (k = 0; k < 3; ++k) if (fabs(w[k] - d[k]) > dev) dev = fabs(w[k] - d[k]);
    return dev;
}

/* Characteristic WENO flux with options: common_alpha = 0 uses the per-field
 * LF speed max|lambda^s| (the reading used everywhere else); 1 uses one speed
 * max(|v_n| + c_f) over the stencil for every field.  *dev (may be NULL)
 * receives the largest deviation of any weight of any field from the linear
 * weights -- the label of a troubled interface. */
static void interface_flux_mode(int z, const double Us[48], double gamma, double eps,
                                int common_alpha, const double *alpha_g, double Fhat[8],
                                double *dev);

void orc_interface_flux_ex(const double Us[48], double gamma, double eps,
                           int common_alpha, double Fhat[8], double *dev)
{
    interface_flux_mode(0, Us, gamma, eps, common_alpha, NULL, Fhat, dev);
}

/* The characteristic flux with the WENO-Z weights (ablation). */
void orc_interface_flux_z(const double Us[48], double gamma, double eps, double Fhat[8])
{
    interface_flux_mode(1, Us, gamma, eps, 0, NULL, Fhat, NULL);
}

/* The characteristic flux with given per-field LF speeds (ablation). */
void orc_interface_flux_alpha(const double Us[48], double gamma, double eps, int z,
                              const double alpha[7], double Fhat[8])
{
    interface_flux_mode(z, Us, gamma, eps, 0, alpha, Fhat, NULL);
}

static void interface_flux_mode(int z, const double Us[48], double gamma, double eps,
                                int common_alpha, const double *alpha_g, double Fhat[8],
                                double *dev)
{
    double F[6][8], lamc[6][8], W[6][8], Wm[8], lam[8], L[64], R[64], Fs[8];
    int j, c, s;
    for (j = 0; j < 6; ++j) {
        const double *U = Us + 8 * j;
        double cf, ca, cs;
        orc_cons_to_prim(U, gamma, W[j]);
        orc_flux(U, 0, gamma, F[j]);
        orc_wave_speeds(U, 0, gamma, &cf, &ca, &cs);
        double vn = W[j][1];
        lamc[j][0] = vn - cf; lamc[j][1] = vn - ca; lamc[j][2] = vn - cs;
        lamc[j][3] = vn;
        lamc[j][4] = vn + cs; lamc[j][5] = vn + ca; lamc[j][6] = vn + cf;
        lamc[j][7] = 0.0;
    }
    for (c = 0; c < 8; ++c) Wm[c] = 0.5 * (W[2][c] + W[3][c]);
    orc_eigensystem(Wm, gamma, lam, L, R);
    double acommon = 0.0, dmax = 0.0;
    for (j = 0; j < 6; ++j) {
        double a = fabs(lamc[j][0] - W[j][1]) + fabs(W[j][1]);   /* c_f + |v_n| */
        if (a > acommon) acommon = a;
    }
    for (s = 0; s < 8; ++s) {
        double fs[6], us[6], alpha = 0.0;
        for (j = 0; j < 6; ++j) {
            double a = 0.0, b = 0.0;
            for (c = 0; c < 8; ++c) {
                a += L[s * 8 + c] * F[j][c];
                b += L[s * 8 + c] * Us[8 * j + c];
            }
            fs[j] = a;
            us[j] = b;
            if (fabs(lamc[j][s]) > alpha) alpha = fabs(lamc[j][s]);
        }
        if (common_alpha && s < 7) alpha = acommon;   /* the B_n identity row keeps 0 */
        if (alpha_g && s < 7) alpha = alpha_g[s];
        Fs[s] = field_flux_mode(z, fs, us, alpha, eps);
        if (dev && s < 7) {
            double dv = weight_deviation(fs, us, alpha, eps);
            if (dv > dmax) dmax = dv;
        }
    }
    if (dev) *dev = dmax;
    for (c = 0; c < 8; ++c) {
        double a = 0.0;
        for (s = 0; s < 8; ++s) a += R[c * 8 + s] * Fs[s];
        Fhat[c] = a;
    }
}

/* Characteristic WENO flux at the interface i+1/2 between Us row 2 and 3. */
void orc_interface_flux(const double Us[48], double gamma, double eps,
                        double Fhat[8])
{
    orc_interface_flux_ex(Us, gamma, eps, 0, Fhat, NULL);
}

/* Linear fifth-order component-wise flux (the cheap flux of interfaces the
 * learned router calls smooth): Lax-Friedrichs split of every conserved
 * component with one speed alpha = max over the stencil of |v_n| + c_f, and
 * the linear-weight form of eq. (1),
 *   F^+: (2, -13, 47, 27, -3)/60 on cells i-2..i+2,
 *   F^-: (-3, 27, 47, -13, 2)/60 on cells i-1..i+3. */
void orc_linear_flux(const double Us[48], double gamma, double Fhat[8])
{
    double F[6][8], alpha = 0.0;
    int j, c;
    for (j = 0; j < 6; ++j) {
        double W[8], cf, ca, cs;
        orc_cons_to_prim(Us + 8 * j, gamma, W);
        orc_flux(Us + 8 * j, 0, gamma, F[j]);
        orc_wave_speeds(Us + 8 * j, 0, gamma, &cf, &ca, &cs);
        if (fabs(W[1]) + cf > alpha) alpha = fabs(W[1]) + cf;
    }
    for (c = 0; c < 8; ++c) {
        double p[6], m[6];
        for (j = 0; j < 6; ++j) {
            p[j] = 0.5 * (F[j][c] + alpha * Us[8 * j + c]);
            m[j] = 0.5 * (F[j][c] - alpha * Us[8 * j + c]);
        }
        Fhat[c] = (2.0 * p[0] - 13.0 * p[1] + 47.0 * p[2] + 27.0 * p[3] - 3.0 * p[4]) / 60.0
                + (-3.0 * m[1] + 27.0 * m[2] + 47.0 * m[3] - 13.0 * m[4] + 2.0 * m[5]) / 60.0;
    }
    Fhat[4] = 0.0;     /* the normal field has no flux */
}

/* ------------------------------------------------------------------------ */
/* Grid helpers.                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n[3], g[3], N[3];
    long sv;                  /* stride between variables */
    double dl[3];
} geom;

static geom mkgeom(const orc_grid *gr)
{
    geom G;
    int d;
    G.n[0] = gr->nx; G.n[1] = gr->ny; G.n[2] = gr->nz;
    G.dl[0] = gr->dx; G.dl[1] = gr->dy; G.dl[2] = gr->dz;
    for (d = 0; d < 3; ++d) {
        G.g[d] = G.n[d] > 1 ? 3 : 0;
        G.N[d] = G.n[d] + 2 * G.g[d];
    }
    G.sv = (long)G.N[0] * G.N[1] * G.N[2];
    return G;
}

static long cidx(const geom *G, int i, int j, int k)
{
    return ((long)(k + G->g[2]) * G->N[1] + (j + G->g[1])) * G->N[0] + (i + G->g[0]);
}

static int active(const geom *G, int d) { return G->n[d] > 1; }

long orc_state_size(const orc_grid *g)
{
    geom G = mkgeom(g);
    return 8 * G.sv;
}

/* Ghost zones, 3 deep (Sec. 2.2): periodic copy or zero-gradient outflow,
 * filled axis by axis so that edges and corners come out consistent. */
void orc_fill_ghosts(const orc_grid *gr, double *u)
{
    geom G = mkgeom(gr);
    int d, v;
    for (d = 0; d < 3; ++d) {
        if (!active(&G, d)) continue;
        int n = G.n[d], g = G.g[d];
        int lo[3], hi[3], e;
        for (e = 0; e < 3; ++e) { lo[e] = -G.g[e]; hi[e] = G.n[e] + G.g[e]; }
        int pos[3];
        for (pos[2] = lo[2]; pos[2] < hi[2]; ++pos[2])
        for (pos[1] = lo[1]; pos[1] < hi[1]; ++pos[1])
        for (pos[0] = lo[0]; pos[0] < hi[0]; ++pos[0]) {
            int x = pos[d];
            if (x >= 0 && x < n) continue;
            int src[3] = { pos[0], pos[1], pos[2] };
            int side = (x < 0) ? 0 : 1;
            int bc = gr->bc[2 * d + side];
            if (bc == 0) src[d] = (x < 0) ? x + n : x - n;
            else         src[d] = (x < 0) ? 0 : n - 1;
            long to = cidx(&G, pos[0], pos[1], pos[2]);
            long from = cidx(&G, src[0], src[1], src[2]);
            for (v = 0; v < 8; ++v) u[v * G.sv + to] = u[v * G.sv + from];
        }
        (void)g;
    }
}

/* Face-flux storage for one sweep direction: faces 0..n along the sweep axis
 * (face f sits at f - 1/2), cells -1..n along each active transverse axis. */
typedef struct {
    int lo[3], cnt[3];
    long total;
    double *f;   /* f[c*total + idx], grid-frame components */
} faces;

static long fidx(const faces *F, int i, int j, int k)
{
    return ((long)(k - F->lo[2]) * F->cnt[1] + (j - F->lo[1])) * F->cnt[0] + (i - F->lo[0]);
}

static double fget(const faces *F, int c, const int pos[3])
{
    return F->f[c * F->total + fidx(F, pos[0], pos[1], pos[2])];
}

/* Edge EMF E_c (Sec. 2.1, constrained transport).  p=(c+1)%3, q=(c+2)%3.
 * The p-flux of B_q equals -E_c and the q-flux of B_p equals +E_c; with both
 * axes active the edge value is the mean of the four adjacent face fluxes. */
static double emf(const geom *G, const faces *FF, int c, int fp, int fq, int cc)
{
    int p = (c + 1) % 3, q = (c + 2) % 3;
    int ap = active(G, p), aq = active(G, q);
    int pos[3];
    if (ap && aq) {
        double t = 0.0;
        pos[c] = cc; pos[p] = fp;
        pos[q] = fq - 1; t -= fget(&FF[p], BX + q, pos);
        pos[q] = fq;     t -= fget(&FF[p], BX + q, pos);
        pos[q] = fq; pos[p] = fp - 1; t += fget(&FF[q], BX + p, pos);
        pos[p] = fp;                  t += fget(&FF[q], BX + p, pos);
        return 0.25 * t;
    }
    if (ap) { pos[c] = cc; pos[p] = fp; pos[q] = 0; return -fget(&FF[p], BX + q, pos); }
    if (aq) { pos[c] = cc; pos[q] = fq; pos[p] = 0; return fget(&FF[q], BX + p, pos); }
    return 0.0;
}

/* Time derivative of the staggered normal field b_n on the n-face fn at
 * transverse cells (j1 along n+1, j2 along n+2): -(curl E)_n. */
static double face_bdot(const geom *G, const faces *FF, int n, int fn, int j1, int j2)
{
    int a1 = (n + 1) % 3, a2 = (n + 2) % 3;
    double r = 0.0;
    if (active(G, a1))
        r -= (emf(G, FF, a2, fn, j1 + 1, j2) - emf(G, FF, a2, fn, j1, j2)) / G->dl[a1];
    if (active(G, a2))
        r += (emf(G, FF, a1, j2 + 1, fn, j1) - emf(G, FF, a1, j2, fn, j1)) / G->dl[a2];
    return r;
}

static int nonphysical(const double U[8], double gamma)
{
    double W[8];
    int v;
    for (v = 0; v < 8; ++v) if (!isfinite(U[v])) return 1;
    orc_cons_to_prim(U, gamma, W);
    return !(W[0] > 0.0) || !(W[7] > 0.0);
}

/* L(U): the semi-discrete right-hand side of one Runge-Kutta stage.
 * Returns 0, or -1 if a stencil cell is non-physical (rho<=0 or p<=0). */
/* Global LF speeds of the d-sweep (ablation of the per-stencil speed): the
 * cells are those the sweep's stencils read; u must hold filled ghosts. */
void orc_lf_global(const orc_grid *gr, const double *u, int d, double alpha[7])
{
    geom G = mkgeom(gr);
    int lo[3], hi[3], e, c, pos[3];
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int perm[8] = { RHO, MX + d, MX + t1, MX + t2, BX + d, BX + t1, BX + t2, EN };
    for (e = 0; e < 3; ++e) {
        if (e == d) { lo[e] = -3; hi[e] = G.n[e] + 3; }
        else if (active(&G, e)) { lo[e] = -1; hi[e] = G.n[e] + 1; }
        else { lo[e] = 0; hi[e] = 1; }
    }
    for (c = 0; c < 7; ++c) alpha[c] = 0.0;
    if (!active(&G, d)) return;                     /* no sweep along an inactive axis */
    for (pos[2] = lo[2]; pos[2] < hi[2]; ++pos[2])
    for (pos[1] = lo[1]; pos[1] < hi[1]; ++pos[1])
    for (pos[0] = lo[0]; pos[0] < hi[0]; ++pos[0]) {
        double U[8], W[8], cf, ca, cs;
        long id = cidx(&G, pos[0], pos[1], pos[2]);
        for (c = 0; c < 8; ++c) U[c] = u[perm[c] * G.sv + id];
        if (nonphysical(U, gr->gamma)) continue;      /* reported by the sweep itself */
        orc_cons_to_prim(U, gr->gamma, W);
        orc_wave_speeds(U, 0, gr->gamma, &cf, &ca, &cs);
        double vn = W[1];
        double lam[7] = { vn - cf, vn - ca, vn - cs, vn, vn + cs, vn + ca, vn + cf };
        for (c = 0; c < 7; ++c)
            if (fabs(lam[c]) > alpha[c]) alpha[c] = fabs(lam[c]);
    }
}

/* Staggered storage (the face-B ablation of the CT reading, Sec. 2.1: CT on a
 * staggered mesh after Ryu et al.): slot B_d of cell i holds the normal field
 * of its lower d-face, i - 1/2.  The cell-centred field the sweeps see is the
 * mean of a cell's two faces; an inactive axis has no faces and its component
 * is used as stored.  The ghosts of u are filled first (the upper face of
 * the last cell is the first ghost's lower face), and those of uc after. */
void orc_face_to_cell(const orc_grid *gr, const double *uin, double *uc)
{
    geom G = mkgeom(gr);
    long ntot = 8 * G.sv;
    double *u = (double *)malloc(sizeof(double) * ntot);
    int pos[3], v, d;
    memcpy(u, uin, sizeof(double) * ntot);
    orc_fill_ghosts(gr, u);
    memcpy(uc, u, sizeof(double) * ntot);
    for (pos[2] = 0; pos[2] < G.n[2]; ++pos[2])
    for (pos[1] = 0; pos[1] < G.n[1]; ++pos[1])
    for (pos[0] = 0; pos[0] < G.n[0]; ++pos[0]) {
        long id = cidx(&G, pos[0], pos[1], pos[2]);
        for (d = 0; d < 3; ++d) {
            if (!active(&G, d)) continue;
            int up[3] = { pos[0], pos[1], pos[2] };
            up[d] += 1;
            v = BX + d;
            uc[v * G.sv + id] = 0.5 * (u[v * G.sv + id] + u[v * G.sv + cidx(&G, up[0], up[1], up[2])]);
        }
    }
    orc_fill_ghosts(gr, uc);
    free(u);
}

void orc_divb_face(const orc_grid *gr, const double *uin, double *max_abs, double *l1)
{
    geom G = mkgeom(gr);
    long ntot = 8 * G.sv, count = 0;
    double *u = (double *)malloc(sizeof(double) * ntot);
    double mx = 0.0, sum = 0.0;
    int pos[3], d;
    memcpy(u, uin, sizeof(double) * ntot);
    orc_fill_ghosts(gr, u);
    for (pos[2] = 0; pos[2] < G.n[2]; ++pos[2])
    for (pos[1] = 0; pos[1] < G.n[1]; ++pos[1])
    for (pos[0] = 0; pos[0] < G.n[0]; ++pos[0]) {
        long id = cidx(&G, pos[0], pos[1], pos[2]);
        double div = 0.0;
        for (d = 0; d < 3; ++d) {
            if (!active(&G, d)) continue;
            int up[3] = { pos[0], pos[1], pos[2] };
            up[d] += 1;
            div += (u[(BX + d) * G.sv + cidx(&G, up[0], up[1], up[2])] - u[(BX + d) * G.sv + id]) / G.dl[d];
        }
        if (fabs(div) > mx) mx = fabs(div);
        sum += fabs(div);
        ++count;
    }
    *max_abs = mx;
    *l1 = count ? sum / count : 0.0;
    free(u);
}

static int rhs_impl(const orc_grid *gr, const double *uin, double *dudt, int fill, int linear)
{
    geom G = mkgeom(gr);
    long ntot = 8 * G.sv;
    double *u = (double *)malloc(sizeof(double) * ntot);
    int bad = 0;
    memcpy(u, uin, sizeof(double) * ntot);
    if (fill) orc_fill_ghosts(gr, u);
    if (gr->b_face) {
        /* the sweeps see the cell-centred state; the face fields are updated
         * below from the same edge EMFs */
        double *uf = (double *)malloc(sizeof(double) * ntot);
        memcpy(uf, u, sizeof(double) * ntot);
        orc_face_to_cell(gr, uf, u);
        free(uf);
    }

    faces FF[3];
    int d, e;
    memset(FF, 0, sizeof FF);
    for (d = 0; d < 3; ++d) {
        if (!active(&G, d)) continue;
        for (e = 0; e < 3; ++e) {
            if (e == d) { FF[d].lo[e] = 0; FF[d].cnt[e] = G.n[e] + 1; }
            else if (active(&G, e)) { FF[d].lo[e] = -1; FF[d].cnt[e] = G.n[e] + 2; }
            else { FF[d].lo[e] = 0; FF[d].cnt[e] = 1; }
        }
        FF[d].total = (long)FF[d].cnt[0] * FF[d].cnt[1] * FF[d].cnt[2];
        FF[d].f = (double *)calloc(8 * FF[d].total, sizeof(double));
    }

    /* Sweeps x, y, z (Sec. 2.2): interface fluxes in the cyclic sweep frame
     * (n, t1, t2) = (d, d+1, d+2), mapped back to grid components. */
    for (d = 0; d < 3; ++d) {
        if (!active(&G, d)) continue;
        int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        int perm[8] = { RHO, MX + d, MX + t1, MX + t2, BX + d, BX + t1, BX + t2, EN };
        int kk;
        double ag[7] = { 0, 0, 0, 0, 0, 0, 0 };
        if (gr->lf_global) orc_lf_global(gr, u, d, ag);
        /* Interfaces are independent: with OpenMP the k-planes are shared
         * among threads (each face is still computed by the same code). */
#pragma omp parallel for schedule(static) reduction(|:bad)
        for (kk = 0; kk < FF[d].cnt[2]; ++kk) {
        int pos[3];
        pos[2] = FF[d].lo[2] + kk;
        for (pos[1] = FF[d].lo[1]; pos[1] < FF[d].lo[1] + FF[d].cnt[1]; ++pos[1])
        for (pos[0] = FF[d].lo[0]; pos[0] < FF[d].lo[0] + FF[d].cnt[0]; ++pos[0]) {
            double Us[48], Fh[8];
            int j, c;
            for (j = 0; j < 6; ++j) {
                int cp[3] = { pos[0], pos[1], pos[2] };
                cp[d] = pos[d] - 3 + j;
                long id = cidx(&G, cp[0], cp[1], cp[2]);
                for (c = 0; c < 8; ++c) Us[8 * j + c] = u[perm[c] * G.sv + id];
                if (nonphysical(Us + 8 * j, gr->gamma)) bad = 1;
            }
            if (linear) orc_linear_flux(Us, gr->gamma, Fh);
            else if (gr->lf_global) orc_interface_flux_alpha(Us, gr->gamma, gr->eps, gr->weights, ag, Fh);
            else if (gr->weights) orc_interface_flux_z(Us, gr->gamma, gr->eps, Fh);
            else orc_interface_flux(Us, gr->gamma, gr->eps, Fh);
            long fi = fidx(&FF[d], pos[0], pos[1], pos[2]);
            for (c = 0; c < 8; ++c) FF[d].f[perm[c] * FF[d].total + fi] = Fh[c];
        }
        }
    }

    /* Flux differences for rho, m, E (x, then y, then z) and CT for B. */
    int kc;
#pragma omp parallel for schedule(static)
    for (kc = 0; kc < G.n[2]; ++kc) {
    int pos[3], dd;
    pos[2] = kc;
    for (pos[1] = 0; pos[1] < G.n[1]; ++pos[1])
    for (pos[0] = 0; pos[0] < G.n[0]; ++pos[0]) {
        long id = cidx(&G, pos[0], pos[1], pos[2]);
        static const int hv[5] = { RHO, MX, MY, MZ, EN };
        int h;
        for (h = 0; h < 5; ++h) {
            double acc = 0.0;
            for (dd = 0; dd < 3; ++dd) {
                if (!active(&G, dd)) continue;
                int pp[3] = { pos[0], pos[1], pos[2] };
                pp[dd] = pos[dd] + 1;
                double fr = fget(&FF[dd], hv[h], pp);
                pp[dd] = pos[dd];
                double fl = fget(&FF[dd], hv[h], pp);
                acc -= (fr - fl) / G.dl[dd];
            }
            dudt[hv[h] * G.sv + id] = acc;
        }
        int n;
        for (n = 0; n < 3; ++n) {
            int a1 = (n + 1) % 3, a2 = (n + 2) % 3;
            double val;
            if (active(&G, n) && gr->b_face)
                val = face_bdot(&G, FF, n, pos[n], pos[a1], pos[a2]);      /* the lower face itself */
            else if (active(&G, n))
                val = 0.5 * (face_bdot(&G, FF, n, pos[n], pos[a1], pos[a2])
                           + face_bdot(&G, FF, n, pos[n] + 1, pos[a1], pos[a2]));
            else
                val = face_bdot(&G, FF, n, 0, pos[a1], pos[a2]);
            dudt[(BX + n) * G.sv + id] = val;
        }
    }
    }

    for (d = 0; d < 3; ++d) free(FF[d].f);
    free(u);
    return bad ? -1 : 0;
}

int orc_rhs(const orc_grid *gr, const double *u, double *dudt)
{
    return rhs_impl(gr, u, dudt, 1, 0);
}

/* As orc_rhs, but the ghost zones of u are used as given (not refilled):
 * L at a cell of a block cut out of a larger state with its ghosts. */
int orc_rhs_nofill(const orc_grid *gr, const double *u, double *dudt)
{
    return rhs_impl(gr, u, dudt, 0, 0);
}

/* As orc_rhs with the linear component-wise flux at every interface. */
int orc_rhs_linear(const orc_grid *gr, const double *u, double *dudt)
{
    return rhs_impl(gr, u, dudt, 1, 1);
}

/* dt = C / max over interior cells of sum_d (|v_d| + c_f,d) / dx_d.
 * Returns a negative value if a cell is non-physical. */
double orc_cfl_dt(const orc_grid *gr, const double *uin)
{
    geom G = mkgeom(gr);
    double smax = 0.0;
    int bad = 0, pos[3], d, v;
    double *ucell = NULL;
    const double *u = uin;
    if (gr->b_face) {                 /* wave speeds of the cell-centred field */
        ucell = (double *)malloc(sizeof(double) * 8 * G.sv);
        orc_face_to_cell(gr, uin, ucell);
        u = ucell;
    }
    for (pos[2] = 0; pos[2] < G.n[2]; ++pos[2])
    for (pos[1] = 0; pos[1] < G.n[1]; ++pos[1])
    for (pos[0] = 0; pos[0] < G.n[0]; ++pos[0]) {
        long id = cidx(&G, pos[0], pos[1], pos[2]);
        double U[8], W[8], sum = 0.0;
        for (v = 0; v < 8; ++v) U[v] = u[v * G.sv + id];
        if (nonphysical(U, gr->gamma)) { bad = 1; continue; }
        orc_cons_to_prim(U, gr->gamma, W);
        for (d = 0; d < 3; ++d) {
            if (!active(&G, d)) continue;
            double cf, ca, cs;
            orc_wave_speeds(U, d, gr->gamma, &cf, &ca, &cs);
            sum += (fabs(W[1 + d]) + cf) / G.dl[d];
        }
        if (sum > smax) smax = sum;
    }
    free(ucell);
    if (bad || !(smax > 0.0)) return -1.0;
    return gr->cfl / smax;
}

/* One classical fourth-order Runge-Kutta step (Sec. 2.1), textbook form:
 * k1..k4 and u + dt/6 (k1 + 2 k2 + 2 k3 + k4).  Ghosts of u are refilled. */
int orc_rk4_step(const orc_grid *gr, double *u, double dt)
{
    long n = orc_state_size(gr), i;
    double *k[4], *tmp = (double *)malloc(sizeof(double) * n);
    int s, bad = 0;
    static const double a[3] = { 0.5, 0.5, 1.0 };
    for (s = 0; s < 4; ++s) k[s] = (double *)calloc(n, sizeof(double));
    memcpy(tmp, u, sizeof(double) * n);
    for (s = 0; s < 4; ++s) {
        if (orc_rhs(gr, tmp, k[s]) != 0) bad = 1;
        if (s < 3) {
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i) tmp[i] = u[i] + a[s] * dt * k[s][i];
        }
    }
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i)
        u[i] = u[i] + dt / 6.0 * (k[0][i] + 2.0 * k[1][i] + 2.0 * k[2][i] + k[3][i]);
    orc_fill_ghosts(gr, u);
    for (s = 0; s < 4; ++s) free(k[s]);
    free(tmp);
    return bad ? -1 : 0;
}

/* SSP-RK3 of Shu & Osher (1988), in its textbook convex-combination form:
 *   u1 = u + dt L(u)
 *   u2 = 3/4 u + 1/4 (u1 + dt L(u1))
 *   u^{n+1} = 1/3 u + 2/3 (u2 + dt L(u2)). */
int orc_ssprk3_step(const orc_grid *gr, double *u, double dt)
{
    long n = orc_state_size(gr), i;
    double *u1 = (double *)malloc(sizeof(double) * n);
    double *u2 = (double *)malloc(sizeof(double) * n);
    double *k = (double *)calloc(n, sizeof(double));
    int bad = 0;
    memcpy(u1, u, sizeof(double) * n);
    if (orc_rhs(gr, u1, k) != 0) bad = 1;               /* L(u) */
    for (i = 0; i < n; ++i) u1[i] = u[i] + dt * k[i];
    if (orc_rhs(gr, u1, k) != 0) bad = 1;
    for (i = 0; i < n; ++i) u2[i] = 0.75 * u[i] + 0.25 * (u1[i] + dt * k[i]);
    if (orc_rhs(gr, u2, k) != 0) bad = 1;
    for (i = 0; i < n; ++i) u[i] = u[i] / 3.0 + 2.0 / 3.0 * (u2[i] + dt * k[i]);
    orc_fill_ghosts(gr, u);
    free(u1); free(u2); free(k);
    return bad ? -1 : 0;
}

/* Neumaier-compensated sums of the 8 conserved variables over the interior. */
void orc_sums(const orc_grid *gr, const double *u, double out[8])
{
    geom G = mkgeom(gr);
    int v, pos[3];
    for (v = 0; v < 8; ++v) {
        double s = 0.0, comp = 0.0;
        for (pos[2] = 0; pos[2] < G.n[2]; ++pos[2])
        for (pos[1] = 0; pos[1] < G.n[1]; ++pos[1])
        for (pos[0] = 0; pos[0] < G.n[0]; ++pos[0]) {
            double x = u[v * G.sv + cidx(&G, pos[0], pos[1], pos[2])];
            double t = s + x;
            if (fabs(s) >= fabs(x)) comp += (s - t) + x;
            else comp += (x - t) + s;
            s = t;
        }
        out[v] = s + comp;
    }
}

/* Corner divergence of the cell-centred field: at each corner, for every
 * active axis d, the mean over the adjacent cell pairs of (B_d(+1)-B_d(0))/dx_d.
 * Corners i+1/2 for i = 0..n-1 on active axes (the last uses a ghost cell). */
void orc_divb(const orc_grid *gr, const double *uin, double *max_abs, double *l1)
{
    geom G = mkgeom(gr);
    long ntot = 8 * G.sv, count = 0;
    double *u = (double *)malloc(sizeof(double) * ntot);
    memcpy(u, uin, sizeof(double) * ntot);
    orc_fill_ghosts(gr, u);
    int nact = 0, d;
    for (d = 0; d < 3; ++d) nact += active(&G, d);
    double mx = 0.0, sum = 0.0;
    int pos[3];
    for (pos[2] = 0; pos[2] < G.n[2]; ++pos[2])
    for (pos[1] = 0; pos[1] < G.n[1]; ++pos[1])
    for (pos[0] = 0; pos[0] < G.n[0]; ++pos[0]) {
        double div = 0.0;
        for (d = 0; d < 3; ++d) {
            if (!active(&G, d)) continue;
            double acc = 0.0;
            int m, nm = 0;
            for (m = 0; m < 8; ++m) {
                int off[3] = { m & 1, (m >> 1) & 1, (m >> 2) & 1 }, e, skip = 0;
                for (e = 0; e < 3; ++e) if (!active(&G, e) && off[e]) skip = 1;
                if (skip || off[d]) continue;
                int c0[3], c1[3];
                for (e = 0; e < 3; ++e) c0[e] = c1[e] = pos[e] + off[e];
                c1[d] += 1;
                acc += u[(BX + d) * G.sv + cidx(&G, c1[0], c1[1], c1[2])]
                     - u[(BX + d) * G.sv + cidx(&G, c0[0], c0[1], c0[2])];
                ++nm;
            }
            div += acc / nm / G.dl[d];
        }
        (void)nact;
        if (fabs(div) > mx) mx = fabs(div);
        sum += fabs(div);
        ++count;
    }
    *max_abs = mx;
    *l1 = count ? sum / count : 0.0;
    free(u);
}

/* Threads of the OpenMP build (the k-plane loops above); the serial build
 * ignores the pragmas and this call.  Returns the thread count in use. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
