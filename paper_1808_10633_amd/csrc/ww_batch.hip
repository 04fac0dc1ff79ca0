// ww_batch.hip -- many independent periodic patches advanced by one
// persistent launch per RK stage.
//
// The patches (arXiv:1808.10633, Sec. 2.2: the domain is cut into patches of
// 18^3-32^3 zones with ghost zones, each computed independently once its
// boundary zones are present) live in one arena.  Resident blocks take whole
// patches, largest first, from a shared counter (one atomic per patch), so a
// block that finishes early takes the next patch and the stage ends when the
// work runs out, not when the unluckiest block does.  A block takes
// each of its patches through the full stage: (stage 0 only) the patch's CFL
// time step (0, and the patch left unadvanced, if any cell is non-physical),
// x/y/z characteristic WENO sweeps into the block's own face-flux scratch
// (y and z first; the flattened x tiles also apply the rho, m, E update),
// then CT and the B part of the RK update -- the same device functions as
// the single-box kernels.  The patches are periodic, and the sweep tiles
// stage each ghost cell from its periodic image: the ghost zones of the
// arena are neither filled nor read.
#include "ww_batch.h"
#include "ww_sweep_dev.h"
#include "ww_update_dev.h"

namespace ww {
namespace {

constexpr int RB = 256;

// CFL time step of one patch (FP64 reduction in fixed order) and its count
// of non-physical cells.
template <typename T>
__device__ __forceinline__ void patch_dt(const T *__restrict__ u, const Geom &G, double gamma,
                                         double cfl, double *dt_out, int32_t *flag_out)
{
    __shared__ double smx[sw::ROWS];
    __shared__ int sfl[sw::ROWS];
    const int tid = threadIdx.x + sw::TILE * threadIdx.y;
    const int ncell = G.n[0] * G.n[1] * G.n[2];     // < 2^31 for edges of at most 1024
    double mx = 0.0;
    int bad = 0;
    // DT_IT cells per thread and pass: all their loads first, then the
    // arithmetic (at two waves per SIMD one cell at a time waits a full
    // memory latency per cell); the maximum and the count do not depend on
    // the order
    constexpr int DT_IT = 4;
    for (int c0 = tid; c0 < ncell; c0 += DT_IT * RB) {
        T w[DT_IT][8];
#pragma unroll
        for (int it = 0; it < DT_IT; ++it) {
            const int c = c0 + it * RB;
            if (c < ncell) {
                int p[3];
                p[0] = c % G.n[0];
                p[1] = (c / G.n[0]) % G.n[1];
                p[2] = c / (G.n[0] * G.n[1]);
                const long id = G.base + p[0] * G.s[0] + p[1] * G.s[1] + (long)p[2] * G.s[2];
#pragma unroll
                for (int v = 0; v < 8; ++v) w[it][v] = u[id + v * G.sv];
            }
        }
#pragma unroll
        for (int it = 0; it < DT_IT; ++it) {
            if (c0 + it * RB >= ncell) continue;
            double q[8];
            bool fin = true;
            for (int v = 0; v < 8; ++v) { q[v] = (double)w[it][v]; fin = fin && isfinite(q[v]); }
            double r = q[0], ir = 1.0 / r;
            double vx = q[1] * ir, vy = q[2] * ir, vz = q[3] * ir;
            double b2 = q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
            double pr = (gamma - 1.0) * (q[7] - 0.5 * (q[1] * vx + q[2] * vy + q[3] * vz) - 0.5 * b2);
            if (!fin || !(r > 0.0) || !(pr > 0.0)) { ++bad; continue; }
            double a2 = gamma * pr * ir;
            double v[3] = { vx, vy, vz };
            double s = 0.0;
            for (int d = 0; d < 3; ++d) {
                double bn2 = q[4 + d] * q[4 + d] * ir;
                double bt2 = b2 * ir - bn2;
                bt2 = bt2 < 0.0 ? 0.0 : bt2;
                double dd = a2 - bn2;
                double cf2 = 0.5 * (a2 + bn2 + bt2 + sqrt(dd * dd + bt2 * (2.0 * a2 + 2.0 * bn2 + bt2)));
                s += (fabs(v[d]) + sqrt(cf2)) * G.idl[d];
            }
            mx = fmax(mx, s);
        }
    }
    // butterfly over the wave's 64 lanes, then the four waves in order
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, m));
        bad += __shfl_xor(bad, m);
    }
    if (threadIdx.x == 0) { smx[threadIdx.y] = mx; sfl[threadIdx.y] = bad; }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < sw::ROWS; ++w) { mx = fmax(mx, smx[w]); bad += sfl[w]; }
        const bool ok = mx > 0.0 && bad == 0;
        *dt_out = ok ? cfl / mx : 0.0;
        *flag_out = bad > 0 ? bad : (ok ? 0 : 1);
    }
    __syncthreads();
}

template <int FT, typename T>
__device__ __forceinline__ void batch_stage(const BatchArgs<T> &a)
{
    constexpr int C0 = sw::tile_cells<0, FT>(), C1 = sw::tile_cells<1, FT>();
    constexpr int CMAX = (C0 > C1 ? C0 : C1) > sw::XF_MAXC ? (C0 > C1 ? C0 : C1) : sw::XF_MAXC;
    __shared__ T sq[sw::NQ * CMAX];
    __shared__ T hx[5 * sw::XF_FACES];     // rho, m, E fluxes of the fused x tile
    __shared__ double sdt;
    const int b = blockIdx.x;
    T *ff = a.scratch + (long)b * a.slot_elems;
    const Phys P = a.P;
    __shared__ int next;
    const int tid0 = threadIdx.x + sw::TILE * threadIdx.y;
    for (;;) {
        if (tid0 == 0) next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int q = next;
        __syncthreads();
        if (q >= a.npatch) break;
        const int p = a.order[q];
        const PatchDesc &D = a.pd[p];
        const Geom G = D.G;
        T *us = a.us + D.soff;
        if (a.s == 0) patch_dt<T>(a.u0 + D.soff, G, P.gamma, a.cfl, &a.dt[p], &a.flag[p]);
        if (threadIdx.x == 0 && threadIdx.y == 0) sdt = a.dt[p];
        __syncthreads();
        const double dtp = sdt;
        __syncthreads();
        if (dtp == 0.0) continue;        // non-physical patch: left unadvanced
        // no ghost fill: the sweep tiles stage ghost cells from their
        // periodic images (WRAP)
        T *fx = ff, *fy = ff + NFC * D.F[0].sc, *fz = fy + NFC * D.F[1].sc;
        // the RK stage of this patch, with its own dt
        StageCoef kc;
        kc.mode = 1;
        kc.s = a.s;
        kc.bdt = a.bw * dtp;
        kc.cdt = a.cw * dtp;
        // y and z sweeps, then the x sweep: on the flattened x tiles it also
        // differences every direction's rho, m, E fluxes and applies their RK
        // update, and the update below is left with constrained transport
        {
            long na, nb;
            sw::sweep_tiles<1, FT>(D.F[1], na, nb);
            for (long tb = 0; tb < nb; ++tb)
                for (long ta = 0; ta < na; ++ta) sw::sweep_tile<1, FT, T, false, false, true, true>(us, fy, G, D.F[1], P, ta, tb, sq);
            sw::sweep_tiles<2, FT>(D.F[2], na, nb);
            for (long tb = 0; tb < nb; ++tb)
                for (long ta = 0; ta < na; ++ta) sw::sweep_tile<2, FT, T, false, false, true, true>(us, fz, G, D.F[2], P, ta, tb, sq);
        }
        const bool fused = D.xflat != 0;
        if (fused) {
            const XFuse<T> xf{ a.u0 + D.soff, a.acc + D.soff, a.acc + D.soff, a.out + D.soff, fy, fz, D.F[1], D.F[2],
                               kc };
            const long total = (long)D.F[0].cnt[0] * D.F[0].cnt[1] * D.F[0].cnt[2];
            const long nt = (total - 1 + sw::XF_FACES - 2) / (sw::XF_FACES - 1);
            for (long t = 0; t < nt; ++t) sw::sweep_tile_xflat_fused<T, true>(us, fx, G, D.F[0], P, t, sq, hx, xf);
        } else {
            long na, nb;
            sw::sweep_tiles<0, FT>(D.F[0], na, nb);
            for (long tb = 0; tb < nb; ++tb)
                for (long ta = 0; ta < na; ++ta) sw::sweep_tile<0, FT, T, false, false, true, true>(us, fx, G, D.F[0], P, ta, tb, sq);
        }
        // flux differences (B only after the fused x sweep), CT, RK
        up::UpdArgs<T> ua;
        ua.u0 = a.u0 + D.soff;
        ua.acc_in = a.acc + D.soff;
        ua.acc_out = a.acc + D.soff;
        ua.out = a.out + D.soff;
        ua.ff[0] = fx; ua.ff[1] = fy; ua.ff[2] = fz;
        ua.fb[0] = D.F[0]; ua.fb[1] = D.F[1]; ua.fb[2] = D.F[2];
        ua.G = G;
        ua.odelta = 0;
        ua.osv = G.sv;
        ua.c = kc;
        ua.c.bonly = fused ? 1 : 0;
        const int tid = threadIdx.x + sw::TILE * threadIdx.y;
        if (fused) {
            // CT and the B stage alone: one thread per (i, j) column segment
            // of up to KSEG cells, marching in k with the z-level EMFs carried
            // (every EMF formed once per column instead of once per adjacent
            // cell, as in update_cell), the next level's loads in flight while
            // a level is computed (two waves per SIMD hide little latency)
            constexpr int KSEG = 16;
            const int nseg = (G.n[2] + KSEG - 1) / KSEG;
            const int ncol = G.n[0] * G.n[1], items = ncol * nseg;     // 32-bit: edges of at most 1024
            for (int t = tid; t < items; t += RB) {
                const int i = t % G.n[0], j = (t / G.n[0]) % G.n[1];
                const int k0 = t / ncol * KSEG;
                up::march_column_b_pipelined<T>(ua, i, j, k0, min(k0 + KSEG, G.n[2]));
            }
        } else {
            // every variable: one thread per cell (marching with the hydro
            // fluxes carried too measured 1.5x slower here: more registers,
            // and whole passes of a small patch's columns half idle)
            const int ncell = G.n[0] * G.n[1] * G.n[2];
            for (int c = tid; c < ncell; c += RB) {
                int pos[3];
                pos[0] = c % G.n[0];
                pos[1] = (c / G.n[0]) % G.n[1];
                pos[2] = c / (G.n[0] * G.n[1]);
                up::update_cell(ua, pos);
            }
        }
        __syncthreads();     // the scratch is reused by the next patch
    }
}

// FP32: at least two waves per SIMD; left to itself the compiler gives the
// 16-faces-per-tile kernel an AGPR past 256 registers and one wave per SIMD.
template <int FT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batch_stage_f32(BatchArgs<float> a)
{
    batch_stage<FT, float>(a);
}

// FP64: from 8 faces per tile on the LDS tile leaves room for one block per
// CU anyway, and at 4 two waves per SIMD would spill.
template <int FT>
__global__ __launch_bounds__(256) void batch_stage_f64(BatchArgs<double> a)
{
    batch_stage<FT, double>(a);
}

template <int FT, typename T> struct StageKernel;
template <int FT> struct StageKernel<FT, float> {
    static constexpr void (*fn)(BatchArgs<float>) = batch_stage_f32<FT>;
};
template <int FT> struct StageKernel<FT, double> {
    static constexpr void (*fn)(BatchArgs<double>) = batch_stage_f64<FT>;
};

template <int FT, typename T>
hipError_t launch_ft(const BatchArgs<T> &a, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL((StageKernel<FT, T>::fn), dim3(nblocks), dim3(sw::TILE, sw::ROWS), 0, st, a);
    return hipGetLastError();
}

}  // namespace

bool batch_xflat_ok(int nx, long nrows) { return nx >= 4 && sw::xflat_cells(nx, nrows) <= sw::XF_MAXC; }

template <typename T>
hipError_t launch_batch_stage(const BatchArgs<T> &a, int ft, int nblocks, hipStream_t st)
{
    switch (ft) {
    case 16: return launch_ft<16, T>(a, nblocks, st);
    case 12: return launch_ft<12, T>(a, nblocks, st);
    case 8: return launch_ft<8, T>(a, nblocks, st);
    default: return launch_ft<4, T>(a, nblocks, st);
    }
}

__global__ void batch_reset_kernel(int32_t *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

hipError_t launch_batch_reset(int32_t *counters, int n, hipStream_t st)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, counters, n);
    return hipGetLastError();
}

template <typename T>
hipError_t batch_occupancy(int ft, int *blocks_per_cu)
{
    switch (ft) {
    case 16: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, StageKernel<16, T>::fn, 256, 0);
    case 12: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, StageKernel<12, T>::fn, 256, 0);
    case 8: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, StageKernel<8, T>::fn, 256, 0);
    default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, StageKernel<4, T>::fn, 256, 0);
    }
}

template hipError_t launch_batch_stage<double>(const BatchArgs<double> &, int, int, hipStream_t);
template hipError_t launch_batch_stage<float>(const BatchArgs<float> &, int, int, hipStream_t);
template hipError_t batch_occupancy<double>(int, int *);
template hipError_t batch_occupancy<float>(int, int *);

}  // namespace ww
