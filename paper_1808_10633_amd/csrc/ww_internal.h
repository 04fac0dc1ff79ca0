// ww_internal.h -- internal types and kernel launchers of the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ww {

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
};
template <typename T>
hipError_t launch_update(const T *u0, const T *acc_in, T *acc_out, T *out, const T *fx,
                         const T *fy, const T *fz, const FaceBox *F, const Geom &G,
                         const StageCoef &c, hipStream_t st);

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
int sums_blocks(const Geom &G);

template <typename T>
hipError_t launch_divb(const T *u, const Geom &G, double *part, int nblk, double *d_out,
                       hipStream_t st);

}  // namespace ww
