// ww_sweep.hip -- launchers of the characteristic WENO5 sweep kernels (one
// tile per block; the device code is in ww_sweep_dev.h).
#include "ww_sweep_dev.h"

namespace ww {
namespace {

template <int DIR, int FT, typename T>
__global__ __launch_bounds__(256) void sweep_kernel(const T *__restrict__ u, T *__restrict__ flux,
                                                     Geom G, FaceBox F, Phys P)
{
    __shared__ T sq[sw::NQ * sw::tile_cells<DIR, FT>()];
    sw::sweep_tile<DIR, FT, T>(u, flux, G, F, P, blockIdx.x, blockIdx.y, sq);
}

template <typename T>
__global__ __launch_bounds__(256) void sweep_xseg_kernel(const T *__restrict__ u, T *__restrict__ flux,
                                                         Geom G, FaceBox F, Phys P)
{
    __shared__ T sq[sw::NQ * sw::ROWS * sw::NCX];
    sw::sweep_tile_xseg<T>(u, flux, G, F, P, blockIdx.x, sq);
}

template <int DIR, int FT, typename T>
hipError_t launch_dir(const T *u, T *flux, const Geom &G, const FaceBox &F, const Phys &P,
                      hipStream_t st)
{
    if (DIR == 0 && F.cnt[0] >= sw::XSEG_MIN) {
        // long rows: flattened face segments, no ragged tile per row
        const long total = (long)F.cnt[0] * F.cnt[1] * F.cnt[2];
        const long nt = (total + sw::TILE * sw::ROWS - 1) / (sw::TILE * sw::ROWS);
        hipLaunchKernelGGL((sweep_xseg_kernel<T>), dim3((unsigned)nt), dim3(sw::TILE, sw::ROWS), 0, st,
                           u, flux, G, F, P);
        return hipGetLastError();
    }
    long na, nb;
    sw::sweep_tiles<DIR, FT>(F, na, nb);
    hipLaunchKernelGGL((sweep_kernel<DIR, FT, T>), dim3((unsigned)na, (unsigned)nb),
                       dim3(sw::TILE, sw::ROWS), 0, st, u, flux, G, F, P);
    return hipGetLastError();
}

// faces per y/z tile: 4 in FP64 (LDS-limited), 8 in FP32
template <typename T> constexpr int ft_of() { return sizeof(T) == 8 ? 4 : 8; }

}  // namespace

template <typename T>
hipError_t launch_sweep(int dir, const T *u, T *flux, const Geom &G, const FaceBox &F,
                        const Phys &P, hipStream_t st)
{
    constexpr int FT = ft_of<T>();
    switch (dir) {
    case 0: return launch_dir<0, FT, T>(u, flux, G, F, P, st);
    case 1: return launch_dir<1, FT, T>(u, flux, G, F, P, st);
    default: return launch_dir<2, FT, T>(u, flux, G, F, P, st);
    }
}

template hipError_t launch_sweep<double>(int, const double *, double *, const Geom &,
                                         const FaceBox &, const Phys &, hipStream_t);
template hipError_t launch_sweep<float>(int, const float *, float *, const Geom &,
                                        const FaceBox &, const Phys &, hipStream_t);

}  // namespace ww
