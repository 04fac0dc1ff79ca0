// ww_sweep.hip -- launchers of the characteristic WENO5 sweep kernels (one
// tile per block; the device code is in ww_sweep_dev.h).
#include "ww_sweep_dev.h"

namespace ww {
namespace {

// At least two waves per SIMD.  The FP64 kernels sit at 248-253 VGPRs; without
// this the WENO-Z instantiations took a few AGPRs more and dropped to one
// wave per SIMD (the x sweep ran 40 % slower).  With it every sweep kernel
// fits in 256 VGPRs without spilling.  The WENO-JS and FP32 code is unchanged
// by it.
#define WW_TWO_WAVES __attribute__((amdgpu_waves_per_eu(2)))

// Hardware block b runs on XCD b % 8 (blocks are dealt round-robin to the
// eight XCDs, each with its own L2).
constexpr int NXCD = 8;

// x sweeps stage the cells' fluxes with the cells (sw::NQ_PRE) in FP32 only:
// the FP32 fused x sweep ran 1.8 % faster at 512^3.  The FP64 sweeps ran 2 %
// slower with them (the larger live set spilled at 256 VGPRs), and the FP32
// y/z tiles lost a block per CU to the larger LDS footprint and ran 5 % slower.
template <typename T> constexpr bool pre_x() { return sizeof(T) == 4; }

// y/z sweeps: tiles (ta: positions of the transverse plane, tb: faces along
// the sweep axis) are renumbered so that each XCD walks whole columns of
// tiles, tb fastest.  A tile's 5 halo rows along the sweep axis were staged
// by the tile before it on the same XCD and come from that XCD's L2.
__device__ __forceinline__ bool column_tile(long ntile, long nb, long per_xcd, int &ta, int &tb)
{
    const long lb = (long)(blockIdx.x % NXCD) * per_xcd + blockIdx.x / NXCD;
    if (lb >= ntile) return false;
    ta = (int)(lb / nb);
    tb = (int)(lb - (long)ta * nb);
    return true;
}

// DIR 0: 2-D grid (ta, tb); DIR 1, 2: 1-D grid in column order.
template <int DIR, int FT, typename T, bool WZ, bool GLF>
__global__ __launch_bounds__(256) WW_TWO_WAVES void sweep_kernel(const T *__restrict__ u, T *__restrict__ flux,
                                                     Geom G, FaceBox F, Phys P, long nb, long ntile,
                                                     long per_xcd)
{
    __shared__ T sq[sw::NQ * sw::tile_cells<DIR, FT>()];
    int ta = blockIdx.x, tb = blockIdx.y;
    if (DIR != 0 && !column_tile(ntile, nb, per_xcd, ta, tb)) return;
    sw::sweep_tile<DIR, FT, T, WZ, GLF>(u, flux, G, F, P, ta, tb, sq);
}

template <typename T, bool WZ, bool GLF>
__global__ __launch_bounds__(256) WW_TWO_WAVES void sweep_xseg_kernel(const T *__restrict__ u, T *__restrict__ flux,
                                                         Geom G, FaceBox F, Phys P)
{
    __shared__ T sq[sw::nq<pre_x<T>()>() * sw::XSEG_CELLS];
    sw::sweep_tile_xseg<T, WZ, GLF, pre_x<T>()>(u, flux, G, F, P, blockIdx.x, sq);
}

// The fused x sweep renumbers blocks so that each XCD walks a contiguous
// range of tiles: neighbouring rows, whose cells read the same y faces, then
// meet in one L2.

template <typename T, bool WZ, bool GLF>
__global__ __launch_bounds__(256) WW_TWO_WAVES void sweep_xfused_kernel(const T *__restrict__ u,
                                                           T *__restrict__ flux, Geom G, FaceBox F, Phys P,
                                                           XFuse<T> xf, long ntile, long per_xcd)
{
    __shared__ T sq[sw::nq<pre_x<T>()>() * sw::XSEG_CELLS];
    __shared__ T hx[5 * sw::TILE * sw::ROWS];
    const long tile = (long)(blockIdx.x % NXCD) * per_xcd + blockIdx.x / NXCD;
    if (tile >= ntile) return;
    sw::sweep_tile_xseg_fused<T, WZ, GLF, pre_x<T>()>(u, flux, G, F, P, tile, sq, hx, xf);
}

template <typename T, bool WZ, bool GLF>
hipError_t launch_xfused(const T *u, T *flux, const Geom &G, const FaceBox &F, const Phys &P, const XFuse<T> &xf,
                         hipStream_t st)
{
    const long total = (long)F.cnt[0] * F.cnt[1] * F.cnt[2];
    const long nt = (total - 1 + sw::XFUSE_STRIDE - 1) / sw::XFUSE_STRIDE;
    const long per = (nt + NXCD - 1) / NXCD;
    hipLaunchKernelGGL((sweep_xfused_kernel<T, WZ, GLF>), dim3((unsigned)(per * NXCD)), dim3(sw::TILE, sw::ROWS), 0,
                       st, u, flux, G, F, P, xf, nt, per);
    return hipGetLastError();
}

// FP64 y/z sweeps: 32 positions x 8 faces per tile (1.6 staged cells per
// face instead of 2.25 with 64 x 4, in 43 KB of LDS); measured 3 % faster at
// 512^3.  FP32 keeps 64 positions x 8 faces (sweep_tile, FT = 8).
constexpr int YZ_PW_F64 = 32;

template <int DIR, int PW, typename T, bool WZ, bool GLF>
__global__ __launch_bounds__(256) WW_TWO_WAVES void sweep_yz_kernel(const T *__restrict__ u, T *__restrict__ flux,
                                                       Geom G, FaceBox F, Phys P, long nb, long ntile,
                                                       long per_xcd)
{
    __shared__ T sq[sw::NQ * sw::yz_cells<PW>()];
    int ta, tb;
    if (!column_tile(ntile, nb, per_xcd, ta, tb)) return;
    sw::sweep_tile_yz<DIR, PW, T, WZ, GLF>(u, flux, G, F, P, ta, tb, sq);
}

template <int DIR, int FT, typename T, bool WZ, bool GLF>
hipError_t launch_dir(const T *u, T *flux, const Geom &G, const FaceBox &F, const Phys &P,
                      hipStream_t st)
{
    if (DIR != 0 && sizeof(T) == 8) {
        constexpr int PW = YZ_PW_F64, B = (DIR == 1) ? 2 : 1;
        const long npos = (long)F.cnt[0] * F.cnt[B];
        const long na = (npos + PW - 1) / PW, nb = (F.cnt[DIR] + 256 / PW - 1) / (256 / PW);
        const long nt = na * nb, per = (nt + NXCD - 1) / NXCD;
        hipLaunchKernelGGL((sweep_yz_kernel<DIR == 0 ? 1 : DIR, PW, T, WZ, GLF>), dim3((unsigned)(per * NXCD)),
                           dim3(sw::TILE, sw::ROWS), 0, st, u, flux, G, F, P, nb, nt, per);
        return hipGetLastError();
    }
    if (DIR == 0 && F.cnt[0] >= sw::XSEG_MIN) {
        // long rows: flattened face segments, no ragged tile per row
        const long total = (long)F.cnt[0] * F.cnt[1] * F.cnt[2];
        const long nt = (total + sw::TILE * sw::ROWS - 1) / (sw::TILE * sw::ROWS);
        hipLaunchKernelGGL((sweep_xseg_kernel<T, WZ, GLF>), dim3((unsigned)nt), dim3(sw::TILE, sw::ROWS), 0, st,
                           u, flux, G, F, P);
        return hipGetLastError();
    }
    long na, nb;
    sw::sweep_tiles<DIR, FT>(F, na, nb);
    if (DIR == 0) {
        hipLaunchKernelGGL((sweep_kernel<DIR, FT, T, WZ, GLF>), dim3((unsigned)na, (unsigned)nb),
                           dim3(sw::TILE, sw::ROWS), 0, st, u, flux, G, F, P, nb, na * nb, 0L);
    } else {
        const long nt = na * nb, per = (nt + NXCD - 1) / NXCD;
        hipLaunchKernelGGL((sweep_kernel<DIR, FT, T, WZ, GLF>), dim3((unsigned)(per * NXCD)),
                           dim3(sw::TILE, sw::ROWS), 0, st, u, flux, G, F, P, nb, nt, per);
    }
    return hipGetLastError();
}

// faces per y/z tile of the FP32 sweep (FP64 y/z sweeps use sweep_yz_kernel)
template <typename T> constexpr int ft_of() { return sizeof(T) == 8 ? 4 : 8; }

template <typename T, bool WZ, bool GLF>
hipError_t launch_dirs(int dir, const T *u, T *flux, const Geom &G, const FaceBox &F, const Phys &P,
                       hipStream_t st)
{
    constexpr int FT = ft_of<T>();
    switch (dir) {
    case 0: return launch_dir<0, FT, T, WZ, GLF>(u, flux, G, F, P, st);
    case 1: return launch_dir<1, FT, T, WZ, GLF>(u, flux, G, F, P, st);
    default: return launch_dir<2, FT, T, WZ, GLF>(u, flux, G, F, P, st);
    }
}

}  // namespace

template <typename T>
hipError_t launch_sweep(int dir, const T *u, T *flux, const Geom &G, const FaceBox &F,
                        const Phys &P, int weights, hipStream_t st)
{
    const bool z = weights == WEIGHTS_Z, glf = P.ag != nullptr;
    if (z && glf) return launch_dirs<T, true, true>(dir, u, flux, G, F, P, st);
    if (z) return launch_dirs<T, true, false>(dir, u, flux, G, F, P, st);
    if (glf) return launch_dirs<T, false, true>(dir, u, flux, G, F, P, st);
    return launch_dirs<T, false, false>(dir, u, flux, G, F, P, st);
}

int sweep_x_fused_min_faces() { return sw::XSEG_MIN; }

template <typename T>
hipError_t launch_sweep_x_fused(const T *u, T *flux, const Geom &G, const FaceBox &F, const Phys &P,
                                int weights, const XFuse<T> &xf, hipStream_t st)
{
    if (F.cnt[0] < sw::XSEG_MIN || !(G.act[0] && G.act[1] && G.act[2])) return hipErrorInvalidValue;
    const bool z = weights == WEIGHTS_Z, glf = P.ag != nullptr;
    if (z && glf) return launch_xfused<T, true, true>(u, flux, G, F, P, xf, st);
    if (z) return launch_xfused<T, true, false>(u, flux, G, F, P, xf, st);
    if (glf) return launch_xfused<T, false, true>(u, flux, G, F, P, xf, st);
    return launch_xfused<T, false, false>(u, flux, G, F, P, xf, st);
}

template hipError_t launch_sweep_x_fused<double>(const double *, double *, const Geom &, const FaceBox &,
                                                 const Phys &, int, const XFuse<double> &, hipStream_t);
template hipError_t launch_sweep_x_fused<float>(const float *, float *, const Geom &, const FaceBox &,
                                                const Phys &, int, const XFuse<float> &, hipStream_t);

template hipError_t launch_sweep<double>(int, const double *, double *, const Geom &,
                                         const FaceBox &, const Phys &, int, hipStream_t);
template hipError_t launch_sweep<float>(int, const float *, float *, const Geom &,
                                        const FaceBox &, const Phys &, int, hipStream_t);

}  // namespace ww
