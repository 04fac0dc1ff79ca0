// ww_aux.hip -- ghost zones, CFL time step and FP64 diagnostics.
//
// Ghost zones (arXiv:1808.10633, Sec. 2.2: 3 cells per side): periodic copy
// or zero-gradient outflow, one launch per axis in the order x, y, z; the
// other axes span their interior (later axes) or their padded range (earlier
// axes) so that edges and corners are consistent.
// CFL: dt = C / max over interior cells of sum_d (|v_d| + c_f,d)/dx_d, in
// FP64, with a count of non-physical cells (rho <= 0, p <= 0, non-finite).
// Global LF speeds (an ablation of the per-stencil speed): per sweep
// direction and field, the largest |lambda^s| over the sweep's cells.
// Reductions are two-pass (per-block partials, then one block) with a fixed
// assignment of cells to threads, wavefront butterflies and a fixed order
// across the waves: results are bitwise reproducible.  No floating-point
// atomics.
#include "ww_internal.h"

#include <math.h>

namespace ww {
namespace {

constexpr int RB = 256;   // reduction block size

template <typename T>
__global__ __launch_bounds__(256) void ghost_kernel(T *__restrict__ u, Geom G, int ax, int bclo,
                                                     int bchi)
{
    const int g = G.g[ax], n = G.n[ax];
    int lo[3], cnt[3];
    for (int e = 0; e < 3; ++e) {
        if (e == ax) { lo[e] = 0; cnt[e] = 2 * g; }
        else if (e < ax) { lo[e] = -G.g[e]; cnt[e] = G.n[e] + 2 * G.g[e]; }
        else { lo[e] = 0; cnt[e] = G.n[e]; }
    }
    const long total = (long)cnt[0] * cnt[1] * cnt[2];
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int pos[3];
    if (total <= 0x7fffffffL) {                 // 32-bit (uniform branch)
        const int ti = (int)t;
        pos[0] = ti % cnt[0];
        pos[1] = (ti / cnt[0]) % cnt[1];
        pos[2] = ti / (cnt[0] * cnt[1]);
    } else {
        pos[0] = (int)(t % cnt[0]);
        pos[1] = (int)((t / cnt[0]) % cnt[1]);
        pos[2] = (int)(t / ((long)cnt[0] * cnt[1]));
    }
    for (int e = 0; e < 3; ++e) pos[e] += lo[e];
    const int gi = pos[ax];
    const bool low = gi < g;
    const int bc = low ? bclo : bchi;
    if (bc == 2) return;                    // user face: filled by the hook
    const int x = low ? gi - g : n + (gi - g);
    int src;
    if (bc == 0) src = low ? x + n : x - n;
    else src = low ? 0 : n - 1;
    int dst[3] = { pos[0], pos[1], pos[2] }, srp[3] = { pos[0], pos[1], pos[2] };
    dst[ax] = x;
    srp[ax] = src;
    const long di = G.base + dst[0] * G.s[0] + dst[1] * G.s[1] + (long)dst[2] * G.s[2];
    const long si = G.base + srp[0] * G.s[0] + srp[1] * G.s[1] + (long)srp[2] * G.s[2];
#pragma unroll
    for (int v = 0; v < 8; ++v) u[di + v * G.sv] = u[si + v * G.sv];
}

// Reductions: a butterfly over the 64 lanes of each wavefront (__shfl_xor,
// every lane ends with the wave's result), then the four waves of a block in
// a fixed order through LDS.  No floating-point atomics: bitwise reproducible.
constexpr int NW = RB / 64;

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ int wave_isum(int v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Block maximum mx, sums sm and fl (valid in thread 0).
__device__ __forceinline__ void block_reduce2(double &mx, double &sm, int &fl)
{
    __shared__ double smx[NW], ssm[NW];
    __shared__ int sfl[NW];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    mx = wave_max(mx);
    sm = wave_sum(sm);
    fl = wave_isum(fl);
    if (l == 0) { smx[w] = mx; ssm[w] = sm; sfl[w] = fl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NW; ++i) { mx = fmax(mx, smx[i]); sm += ssm[i]; fl += sfl[i]; }
    }
}

// Block reduction of K values per thread (sum or max; valid in thread 0).
template <int K, bool MAX>
__device__ __forceinline__ void block_reduce_k(double (&v)[K])
{
    __shared__ double sv[K][NW];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = MAX ? wave_max(v[k]) : wave_sum(v[k]);
        if (l == 0) sv[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k)
            for (int i = 1; i < NW; ++i) v[k] = MAX ? fmax(v[k], sv[k][i]) : v[k] + sv[k][i];
}

// Cell c of the interior in row-major order.  32-bit arithmetic whenever the
// box has fewer than 2^31 cells (every box that fits in memory: a 64-bit
// division is a long software sequence on the GPU); the branch is uniform.
__device__ __forceinline__ void cell_pos(const Geom &G, long c, int (&p)[3])
{
    if ((long)G.n[0] * G.n[1] * G.n[2] <= 0x7fffffffL) {
        const int ci = (int)c;
        p[0] = ci % G.n[0];
        p[1] = (ci / G.n[0]) % G.n[1];
        p[2] = ci / (G.n[0] * G.n[1]);
        return;
    }
    p[0] = (int)(c % G.n[0]);
    p[1] = (int)((c / G.n[0]) % G.n[1]);
    p[2] = (int)(c / ((long)G.n[0] * G.n[1]));
}

template <typename T>
__global__ __launch_bounds__(RB) void cfl_partial(const T *__restrict__ u, Geom G, double gamma,
                                                   double *part, int32_t *partflag)
{
    const long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    double mx = 0.0, dummy = 0.0;
    int bad = 0;
    for (long c = (long)blockIdx.x * RB + threadIdx.x; c < ncell; c += (long)gridDim.x * RB) {
        int p[3];
        cell_pos(G, c, p);
        const long id = G.base + p[0] * G.s[0] + p[1] * G.s[1] + (long)p[2] * G.s[2];
        double q[8];
        bool fin = true;
        for (int v = 0; v < 8; ++v) { q[v] = (double)u[id + v * G.sv]; fin = fin && isfinite(q[v]); }
        double r = q[0];
        double ir = 1.0 / r;
        double vx = q[1] * ir, vy = q[2] * ir, vz = q[3] * ir;
        double b2 = q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
        double pr = (gamma - 1.0) * (q[7] - 0.5 * (q[1] * vx + q[2] * vy + q[3] * vz) - 0.5 * b2);
        if (!fin || !(r > 0.0) || !(pr > 0.0)) { ++bad; continue; }
        double a2 = gamma * pr * ir;
        double v[3] = { vx, vy, vz };
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (!G.act[d]) continue;
            double bn2 = q[4 + d] * q[4 + d] * ir;
            double bt2 = b2 * ir - bn2;
            bt2 = bt2 < 0.0 ? 0.0 : bt2;
            double dd = a2 - bn2;
            double cf2 = 0.5 * (a2 + bn2 + bt2 + sqrt(dd * dd + bt2 * (2.0 * a2 + 2.0 * bn2 + bt2)));
            s += (fabs(v[d]) + sqrt(cf2)) * G.idl[d];
        }
        mx = fmax(mx, s);
    }
    block_reduce2(mx, dummy, bad);
    if (threadIdx.x == 0) { part[blockIdx.x] = mx; partflag[blockIdx.x] = bad; }
}

__global__ __launch_bounds__(RB) void cfl_final(const double *part, const int32_t *partflag, int nblk,
                                                 double cfl, double *d_dt, int32_t *d_flag)
{
    double mx = 0.0, dummy = 0.0;
    int bad = 0;
    for (int b = threadIdx.x; b < nblk; b += RB) { mx = fmax(mx, part[b]); bad += partflag[b]; }
    block_reduce2(mx, dummy, bad);
    if (threadIdx.x == 0) {
        *d_dt = (mx > 0.0) ? cfl / mx : 0.0;
        *d_flag = (mx > 0.0) ? bad : (bad > 0 ? bad : 1);
    }
}

// Global LF speeds of the d-sweep: per-block maxima of the seven |lambda^s|
// over a fixed grid-stride assignment of the sweep's cell set.
template <typename T>
__global__ __launch_bounds__(RB) void lf_partial(const T *__restrict__ u, Geom G, int d, double gamma,
                                                 double *part)
{
    int lo[3], cnt[3];
    for (int e = 0; e < 3; ++e) {
        if (e == d) { lo[e] = -G.g[e]; cnt[e] = G.n[e] + 2 * G.g[e]; }
        else if (G.act[e]) { lo[e] = -1; cnt[e] = G.n[e] + 2; }
        else { lo[e] = 0; cnt[e] = 1; }
    }
    const long total = (long)cnt[0] * cnt[1] * cnt[2];
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    double m[7] = { 0, 0, 0, 0, 0, 0, 0 };
    for (long c = (long)blockIdx.x * RB + threadIdx.x; c < total; c += (long)gridDim.x * RB) {
        int p0, p1, p2;
        if (total <= 0x7fffffffL) {             // 32-bit (uniform branch)
            const int ci = (int)c;
            p0 = lo[0] + ci % cnt[0];
            p1 = lo[1] + (ci / cnt[0]) % cnt[1];
            p2 = lo[2] + ci / (cnt[0] * cnt[1]);
        } else {
            p0 = lo[0] + (int)(c % cnt[0]);
            p1 = lo[1] + (int)((c / cnt[0]) % cnt[1]);
            p2 = lo[2] + (int)(c / ((long)cnt[0] * cnt[1]));
        }
        const long id = G.base + p0 * G.s[0] + p1 * G.s[1] + (long)p2 * G.s[2];
        double q[8];
        bool fin = true;
        for (int v = 0; v < 8; ++v) { q[v] = (double)u[id + v * G.sv]; fin = fin && isfinite(q[v]); }
        const double r = q[0];
        const double ir = 1.0 / r;
        const double b2 = q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
        const double pr = (gamma - 1.0) * (q[7] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * ir - 0.5 * b2);
        if (!fin || !(r > 0.0) || !(pr > 0.0)) continue;
        const double vn = q[1 + d] * ir;
        const double a2 = gamma * pr * ir;
        const double bn2 = q[4 + d] * q[4 + d] * ir;
        double bt2 = (q[4 + t1] * q[4 + t1] + q[4 + t2] * q[4 + t2]) * ir;
        const double dd = a2 - bn2;
        const double cf2 = 0.5 * (a2 + bn2 + bt2 + sqrt(dd * dd + bt2 * (2.0 * a2 + 2.0 * bn2 + bt2)));
        const double cf = sqrt(cf2), cs = sqrt(a2 * bn2 / cf2), ca = sqrt(bn2);
        const double lam[7] = { vn - cf, vn - ca, vn - cs, vn, vn + cs, vn + ca, vn + cf };
        for (int k = 0; k < 7; ++k) m[k] = fmax(m[k], fabs(lam[k]));
    }
    block_reduce_k<7, true>(m);
    if (threadIdx.x == 0)
        for (int k = 0; k < 7; ++k) part[7 * blockIdx.x + k] = m[k];
}

__global__ __launch_bounds__(RB) void lf_final(const double *part, int nblk, double *out)
{
    double m[7] = { 0, 0, 0, 0, 0, 0, 0 };
    for (int b = threadIdx.x; b < nblk; b += RB)
        for (int k = 0; k < 7; ++k) m[k] = fmax(m[k], part[7 * b + k]);
    block_reduce_k<7, true>(m);
    if (threadIdx.x == 0)
        for (int k = 0; k < 7; ++k) out[k] = m[k];
}

template <typename T>
__global__ __launch_bounds__(RB) void sums_partial(const T *__restrict__ u, Geom G, double *part)
{
    const long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    double acc[8] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    for (long c = (long)blockIdx.x * RB + threadIdx.x; c < ncell; c += (long)gridDim.x * RB) {
        int p[3];
        cell_pos(G, c, p);
        const long id = G.base + p[0] * G.s[0] + p[1] * G.s[1] + (long)p[2] * G.s[2];
        for (int v = 0; v < 8; ++v) acc[v] += (double)u[id + v * G.sv];
    }
    block_reduce_k<8, false>(acc);
    if (threadIdx.x == 0)
        for (int v = 0; v < 8; ++v) part[blockIdx.x * 8 + v] = acc[v];
}

__global__ __launch_bounds__(RB) void sums_final(const double *part, int nblk, double *out)
{
    double acc[8] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    for (int b = threadIdx.x; b < nblk; b += RB)
        for (int v = 0; v < 8; ++v) acc[v] += part[b * 8 + v];
    block_reduce_k<8, false>(acc);
    if (threadIdx.x == 0)
        for (int v = 0; v < 8; ++v) out[v] = acc[v];
}

// Corner divergence at corners i+1/2 (i = 0..n-1) on active axes.
template <typename T>
__global__ __launch_bounds__(RB) void divb_partial(const T *__restrict__ u, Geom G, double *part)
{
    const long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    double mx = 0.0, sm = 0.0;
    int dummy = 0;
    for (long c = (long)blockIdx.x * RB + threadIdx.x; c < ncell; c += (long)gridDim.x * RB) {
        int p[3];
        cell_pos(G, c, p);
        double div = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (!G.act[d]) continue;
            double acc = 0.0;
            int nm = 0;
            for (int m = 0; m < 8; ++m) {
                int off[3] = { m & 1, (m >> 1) & 1, (m >> 2) & 1 };
                bool skip = off[d] != 0;
                for (int e = 0; e < 3; ++e) skip = skip || (!G.act[e] && off[e]);
                if (skip) continue;
                long i0 = G.base + (p[0] + off[0]) * G.s[0] + (p[1] + off[1]) * G.s[1]
                        + (long)(p[2] + off[2]) * G.s[2];
                long i1 = i0 + G.s[d];
                acc += (double)u[i1 + (4 + d) * G.sv] - (double)u[i0 + (4 + d) * G.sv];
                ++nm;
            }
            div += acc / nm * G.idl[d];
        }
        mx = fmax(mx, fabs(div));
        sm += fabs(div);
    }
    block_reduce2(mx, sm, dummy);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = mx; part[2 * blockIdx.x + 1] = sm; }
}

__global__ __launch_bounds__(RB) void divb_final(const double *part, int nblk, double ncell,
                                                  double *out)
{
    double mx = 0.0, sm = 0.0;
    int dummy = 0;
    for (int b = threadIdx.x; b < nblk; b += RB) { mx = fmax(mx, part[2 * b]); sm += part[2 * b + 1]; }
    block_reduce2(mx, sm, dummy);
    if (threadIdx.x == 0) { out[0] = mx; out[1] = sm / ncell; }
}

// Staggered storage (periodic boxes): cell-centred state of the interior cells.
template <typename T>
__global__ __launch_bounds__(RB) void face_to_cell_kernel(const T *__restrict__ u, T *__restrict__ uc, Geom G)
{
    const long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    const long c = (long)blockIdx.x * RB + threadIdx.x;
    if (c >= ncell) return;
    int p[3];
    cell_pos(G, c, p);
    const long id = G.base + p[0] * G.s[0] + p[1] * G.s[1] + (long)p[2] * G.s[2];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int d = v - 4;
        // the upper face of the last cell is the periodic image of face 0
        if (d >= 0 && d < 3 && G.act[d])
            uc[id + v * G.sv] = T(0.5) * (u[id + v * G.sv]
                                          + u[id + (p[d] + 1 < G.n[d] ? G.s[d] : -(long)(G.n[d] - 1) * G.s[d])
                                              + v * G.sv]);
        else
            uc[id + v * G.sv] = u[id + v * G.sv];
    }
}

// Face divergence of a staggered state (periodic box).
template <typename T>
__global__ __launch_bounds__(RB) void divb_face_partial(const T *__restrict__ u, Geom G, double *part)
{
    const long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    double mx = 0.0, sm = 0.0;
    int dummy = 0;
    for (long c = (long)blockIdx.x * RB + threadIdx.x; c < ncell; c += (long)gridDim.x * RB) {
        int p[3];
        cell_pos(G, c, p);
        const long id = G.base + p[0] * G.s[0] + p[1] * G.s[1] + (long)p[2] * G.s[2];
        double div = 0.0;
        for (int d = 0; d < 3; ++d)
            if (G.act[d]) {
                const long up = p[d] + 1 < G.n[d] ? G.s[d] : -(long)(G.n[d] - 1) * G.s[d];   // periodic
                div += ((double)u[id + up + (4 + d) * G.sv] - (double)u[id + (4 + d) * G.sv]) * G.idl[d];
            }
        mx = fmax(mx, fabs(div));
        sm += fabs(div);
    }
    block_reduce2(mx, sm, dummy);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = mx; part[2 * blockIdx.x + 1] = sm; }
}

}  // namespace

void box_geom(const int n[3], const double dl[3], Geom &G, FaceBox F[3])
{
    int N[3];
    for (int d = 0; d < 3; ++d) {
        G.n[d] = n[d];
        G.act[d] = n[d] > 1;
        G.g[d] = G.act[d] ? 3 : 0;
        G.dl[d] = dl[d];
        G.idl[d] = 1.0 / dl[d];
        N[d] = n[d] + 2 * G.g[d];
    }
    G.s[0] = 1;
    G.s[1] = N[0];
    G.s[2] = (long)N[0] * N[1];
    G.sv = (long)N[0] * N[1] * N[2];
    G.base = G.g[0] + G.g[1] * G.s[1] + G.g[2] * G.s[2];
    for (int d = 0; d < 3; ++d) {
        FaceBox &B = F[d];
        for (int e = 0; e < 3; ++e) {
            if (e == d) { B.lo[e] = 0; B.cnt[e] = n[e] + 1; }
            else if (G.act[e]) { B.lo[e] = -1; B.cnt[e] = n[e] + 2; }
            else { B.lo[e] = 0; B.cnt[e] = 1; }
        }
        B.s[0] = 1;
        B.s[1] = B.cnt[0];
        B.s[2] = (long)B.cnt[0] * B.cnt[1];
        B.sc = (long)B.cnt[0] * B.cnt[1] * B.cnt[2];
    }
}

int cfl_blocks(const Geom &G)
{
    long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    long b = (ncell + RB - 1) / RB;
    return (int)(b < 2048 ? b : 2048);
}
int sums_blocks(const Geom &G) { return cfl_blocks(G); }

template <typename T>
hipError_t launch_ghosts(T *u, const Geom &G, int axis, const int bc[6], hipStream_t st)
{
    if (!G.act[axis]) return hipSuccess;
    long total = 2L * G.g[axis];
    for (int e = 0; e < 3; ++e) {
        if (e == axis) continue;
        total *= (e < axis) ? (G.n[e] + 2 * G.g[e]) : G.n[e];
    }
    dim3 grd((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL((ghost_kernel<T>), grd, dim3(256), 0, st, u, G, axis, bc[2 * axis],
                       bc[2 * axis + 1]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cfl(const T *u, const Geom &G, double gamma, double cfl, double *part,
                      int32_t *partflag, int nblk, double *d_dt, int32_t *d_flag, hipStream_t st)
{
    hipLaunchKernelGGL((cfl_partial<T>), dim3(nblk), dim3(RB), 0, st, u, G, gamma, part, partflag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cfl_final, dim3(1), dim3(RB), 0, st, part, partflag, nblk, cfl, d_dt, d_flag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lf_global(const T *u, const Geom &G, int d, double gamma, double *part, double *d_out,
                            hipStream_t st)
{
    if (!G.act[d]) return hipSuccess;
    long total = 1;
    for (int e = 0; e < 3; ++e)
        total *= (e == d) ? G.n[e] + 2 * G.g[e] : (G.act[e] ? G.n[e] + 2 : 1);
    const long b = (total + RB - 1) / RB;
    const int nblk = (int)(b < LF_BLOCKS ? b : LF_BLOCKS);
    hipLaunchKernelGGL((lf_partial<T>), dim3(nblk), dim3(RB), 0, st, u, G, d, gamma, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lf_final, dim3(1), dim3(RB), 0, st, part, nblk, d_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sums(const T *u, const Geom &G, double *part, int nblk, double *d_out,
                       hipStream_t st)
{
    hipLaunchKernelGGL((sums_partial<T>), dim3(nblk), dim3(RB), 0, st, u, G, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sums_final, dim3(1), dim3(RB), 0, st, part, nblk, d_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_divb(const T *u, const Geom &G, double *part, int nblk, double *d_out,
                       hipStream_t st)
{
    hipLaunchKernelGGL((divb_partial<T>), dim3(nblk), dim3(RB), 0, st, u, G, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double ncell = (double)G.n[0] * G.n[1] * G.n[2];
    hipLaunchKernelGGL(divb_final, dim3(1), dim3(RB), 0, st, part, nblk, ncell, d_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_face_to_cell(const T *u, T *uc, const Geom &G, hipStream_t st)
{
    const long ncell = (long)G.n[0] * G.n[1] * G.n[2];
    hipLaunchKernelGGL((face_to_cell_kernel<T>), dim3((unsigned)((ncell + RB - 1) / RB)), dim3(RB), 0, st, u, uc, G);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_divb_face(const T *u, const Geom &G, double *part, int nblk, double *d_out, hipStream_t st)
{
    hipLaunchKernelGGL((divb_face_partial<T>), dim3(nblk), dim3(RB), 0, st, u, G, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double ncell = (double)G.n[0] * G.n[1] * G.n[2];
    hipLaunchKernelGGL(divb_final, dim3(1), dim3(RB), 0, st, part, nblk, ncell, d_out);
    return hipGetLastError();
}

#define WW_INST(T)                                                                           \
    template hipError_t launch_ghosts<T>(T *, const Geom &, int, const int *, hipStream_t);  \
    template hipError_t launch_cfl<T>(const T *, const Geom &, double, double, double *,      \
                                      int32_t *, int, double *, int32_t *, hipStream_t);     \
    template hipError_t launch_sums<T>(const T *, const Geom &, double *, int, double *,      \
                                       hipStream_t);                                         \
    template hipError_t launch_divb<T>(const T *, const Geom &, double *, int, double *,      \
                                       hipStream_t);                                         \
    template hipError_t launch_lf_global<T>(const T *, const Geom &, int, double, double *,   \
                                            double *, hipStream_t);                          \
    template hipError_t launch_face_to_cell<T>(const T *, T *, const Geom &, hipStream_t);    \
    template hipError_t launch_divb_face<T>(const T *, const Geom &, double *, int, double *, \
                                            hipStream_t);
WW_INST(double)
WW_INST(float)

}  // namespace ww
