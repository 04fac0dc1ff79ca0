// ww_internal.h -- internal types and kernel launchers of the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/wombat_weno.h"

namespace ww {

// Every device and pinned-host allocation of the library goes through these
// two functions, which count them (wombat_weno_alloc_count) and honour the
// WOMBAT_WENO_FAIL_ALLOC test hook (the k-th allocation after the latest
// init or batch init fails).
hipError_t dev_alloc(void **p, size_t bytes);
hipError_t host_alloc(void **p, size_t bytes);
void alloc_hook_reset();
long long alloc_total();

// Geometry of one padded state array (u[v][k][j][i], i fastest).
struct Geom {
    int n[3];          // interior cells per axis
    int g[3];          // ghost cells per side (3 on active axes, 0 otherwise)
    int act[3];        // axis active (n > 1)
    long s[3];         // element strides of i, j, k
    long sv;           // stride between variables
    long base;         // element index of cell (0,0,0)
    double dl[3];      // cell widths
    double idl[3];     // 1 / cell widths
};

// Face-flux box of one sweep direction d: faces 0..n_d along d (face f sits
// at f - 1/2), cells -1..n along active transverse axes, 0 on inactive ones.
// Components: 0 rho, 1 mx, 2 my, 3 mz, 4 B_(d+1)%3, 5 B_(d+2)%3, 6 E.
struct FaceBox {
    int lo[3], cnt[3];
    long s[3];         // strides within one component
    long sc;           // stride between components
    __host__ __device__ long idx(int i, int j, int k) const {
        return (long)(i - lo[0]) * s[0] + (long)(j - lo[1]) * s[1] + (long)(k - lo[2]) * s[2];
    }
};
constexpr int NFC = 7;   // stored face-flux components

// Geometry of a box of n[3] interior cells of widths dl[3] (an axis with
// n == 1 is inactive) and its three face boxes.
void box_geom(const int n[3], const double dl[3], Geom &G, FaceBox F[3]);

// Checks of a configuration shared by every entry point that takes one:
// WW_OK or WW_ERR_INVALID_ARG with the reason in why.
int validate_config(const wombat_weno_config *c, std::string &why);
// Message of a failure without a context (wombat_weno_last_error(NULL)).
void set_global_error(const std::string &msg);

struct Phys {
    double gamma, eps;
    double igm1;       // 1 / (gamma - 1)
    const double *ag = nullptr;   // global LF speeds of this sweep (7 fields), or null
};

// Launchers (return the hipError_t of the launch).
// weights: WEIGHTS_JS (eq. (3)-(5)) or WEIGHTS_Z (Borges et al. 2008).
constexpr int WEIGHTS_JS = 0, WEIGHTS_Z = 1;
template <typename T>
hipError_t launch_sweep(int dir, const T *u, T *flux, const Geom &G, const FaceBox &F,
                        const Phys &P, int weights, hipStream_t st);

// mode 0: out = L(U); mode 1: low-storage classical RK4 stage s (acc and
// out as below); mode 2: convex-combination stage of SSP-RK3,
// out = a0 u0 + a1 us + cdt L(us), with us passed as acc_in (read only if
// a1 != 0).
struct StageCoef {
    int mode;          // 0 rhs, 1 RK4 stage, 2 SSP-RK3 stage
    int s;             // 0..3
    double bdt;        // weight of L in acc (mode 1)
    double cdt;        // weight of L in out
    double a0 = 0.0;   // mode 2: weight of u0
    double a1 = 0.0;   // mode 2: weight of us
    int bonly = 0;     // update B only (CT): rho, m, E were updated by the fused x sweep
    int stag = 0;      // staggered storage: B slot d of a cell is its lower d-face's field,
                       // advanced by that face's update (not the mean of two faces)
};
// odelta, osv: out[v] of the cell at state index id is written at
// out[id + odelta + v * osv] (defaults: the layout of the other arrays).
template <typename T>
hipError_t launch_update(const T *u0, const T *acc_in, T *acc_out, T *out, const T *fx,
                         const T *fy, const T *fz, const FaceBox *F, const Geom &G,
                         const StageCoef &c, hipStream_t st, long odelta = 0, long osv = 0);

// The x sweep with the rho, m, E part of the update fused in (3 active axes,
// rows of at least sweep_x_fused_min_faces() faces): per interior cell, the
// x flux difference from the sweep's own face fluxes, the y and z flux
// differences from the face fluxes of those sweeps (fy, fz in their boxes),
// in the order x, y, z, then the RK combination of the stage for those five
// variables.  Only the transverse-B components (slots 4, 5) of the x fluxes
// are stored; the update then runs with StageCoef::bonly.
template <typename T>
struct XFuse {
    const T *u0;
    const T *acc_in;
    T *acc_out;
    T *out;
    const T *fy, *fz;
    FaceBox by, bz;
    StageCoef c;
};
template <typename T>
hipError_t launch_sweep_x_fused(const T *u, T *flux, const Geom &G, const FaceBox &F, const Phys &P,
                                int weights, const XFuse<T> &xf, hipStream_t st);
int sweep_x_fused_min_faces();

template <typename T>
hipError_t launch_ghosts(T *u, const Geom &G, int axis, const int bc[6], hipStream_t st);

// CFL reduction: writes partial maxima / flags to scratch, then dt to d_dt.
template <typename T>
hipError_t launch_cfl(const T *u, const Geom &G, double gamma, double cfl, double *part,
                      int32_t *partflag, int nblk, double *d_dt, int32_t *d_flag,
                      hipStream_t st);
int cfl_blocks(const Geom &G);

// Global LF speeds of the d-sweep (the LF-speed ablation): per field, the
// largest |lambda^s| over the cells the sweep's stencils read (3-deep ghosts
// along d, one transverse ghost layer on active transverse axes), in FP64;
// non-physical cells are skipped (the CFL reduction reports them).  part
// holds LF_PART_DOUBLES; d_out receives 7 doubles.
constexpr int LF_BLOCKS = 1024;
constexpr long LF_PART_DOUBLES = 7L * LF_BLOCKS;
template <typename T>
hipError_t launch_lf_global(const T *u, const Geom &G, int d, double gamma, double *part, double *d_out,
                            hipStream_t st);

template <typename T>
hipError_t launch_sums(const T *u, const Geom &G, double *part, int nblk, double *d_out,
                       hipStream_t st);

// Staggered storage (periodic boxes): the cell-centred state uc of u
// (interior; B_d the mean of a cell's two d-faces on an active axis, the
// slot itself on an inactive one), and the face divergence
// sum_d (b_d(i+1/2) - b_d(i-1/2))/dx_d of u (max, mean of |.|) into d_out[0..1].
template <typename T>
hipError_t launch_face_to_cell(const T *u, T *uc, const Geom &G, hipStream_t st);
template <typename T>
hipError_t launch_divb_face(const T *u, const Geom &G, double *part, int nblk, double *d_out,
                            hipStream_t st);
int sums_blocks(const Geom &G);

template <typename T>
hipError_t launch_divb(const T *u, const Geom &G, double *part, int nblk, double *d_out,
                       hipStream_t st);

}  // namespace ww
