// ww_router.hip -- the learned troubled-interface router.
//
// An MLP 48 -> 32 -> 32 -> 1 (ReLU, sigmoid) reads the normalised six-cell
// stencil of an interface and predicts whether the full characteristic WENO
// flux (arXiv:1808.10633 Sec. 2.1) is needed there, i.e. whether some WENO
// weight departs from its linear value by more than 1e-2.  Interfaces called
// smooth take the linear fifth-order component-wise flux instead.
//
// Matrix products run on MFMA (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32
// accumulation).  Layers are computed transposed, Z^T = W X^T, so that the
// output registers of one layer (lane l holds rows 4(l/16)+i, column l%16 of
// a 16x16 tile) are exactly the B operand of the next layer: no shuffles.
// Parameters are one FP32 vector of 2657 values: W1 (32x48, [out][in]), b1,
// W2 (32x32), b2, w3 (32), b3; BF16 copies are made per block.
#include "ww_router.h"
#include "ww_sweep_dev.h"

namespace ww {
namespace rt {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int OW1 = 0, OB1 = 1536, OW2 = 1568, OB2 = 2592, OW3 = 2624, OB3 = 2656;
constexpr int XS = 52;     // LDS row stride (BF16 elements) of the feature matrix

__device__ __forceinline__ short f2bf(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);      // round to nearest even
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf2f(short h)
{
    return __uint_as_float(((unsigned)(unsigned short)h) << 16);
}

// The MLP in MFMA operand layout for this lane (l = lane, r = l%16, q = l/16).
struct MlpRegs {
    bf4 a1[2][3];                  // A of layer 1, tile (ot, kt): W1[16ot+r][16kt+4q+i]
    bf4 a2[2][2];                  // A of layer 2, tile (ot, kt): W2[16ot+r][16kt+4q+i]
    float b1[2][4], b2[2][4], w3[2][4];   // entries of output rows 16ot+4q+i
    float b3;
};

__device__ __forceinline__ void load_mlp(const float *__restrict__ th, MlpRegs &R)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {
#pragma unroll
        for (int kt = 0; kt < 3; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) R.a1[ot][kt][i] = f2bf(th[OW1 + (16 * ot + r) * NIN + 16 * kt + 4 * q + i]);
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) R.a2[ot][kt][i] = f2bf(th[OW2 + (16 * ot + r) * NH + 16 * kt + 4 * q + i]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            R.b1[ot][i] = th[OB1 + 16 * ot + 4 * q + i];
            R.b2[ot][i] = th[OB2 + 16 * ot + 4 * q + i];
            R.w3[ot][i] = th[OW3 + 16 * ot + 4 * q + i];
        }
    }
    R.b3 = th[OB3];
}

// Forward pass of the 64 samples of this wave, rows xs[m*XS + k] (BF16),
// m = 0..63.  lg[st] receives the logit of sample 16*st + l%16.  If a1s/a2s
// are given, the pre-activations (with bias) are stored there as [m][32].
__device__ __forceinline__ void mlp_wave(const short *xs, const MlpRegs &R, float (&lg)[4],
                                         float *a1s, float *a2s)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int m = 16 * st + r;
        f4 z1[2] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
#pragma unroll
        for (int kt = 0; kt < 3; ++kt) {
            const bf4 bx = *(const bf4 *)(xs + m * XS + 16 * kt + 4 * q);
#pragma unroll
            for (int ot = 0; ot < 2; ++ot)
                z1[ot] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a1[ot][kt], bx, z1[ot], 0, 0, 0);
        }
        bf4 h1[2];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float a = z1[ot][i] + R.b1[ot][i];
                if (a1s) a1s[(16 * st + r) * NH + 16 * ot + 4 * q + i] = a;
                h1[ot][i] = f2bf(fmaxf(a, 0.f));
            }
        f4 z2[2] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int ot = 0; ot < 2; ++ot)
                z2[ot] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a2[ot][kt], h1[kt], z2[ot], 0, 0, 0);
        float part = 0.f;
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float a = z2[ot][i] + R.b2[ot][i];
                if (a2s) a2s[(16 * st + r) * NH + 16 * ot + 4 * q + i] = a;
                part += R.w3[ot][i] * fmaxf(a, 0.f);
            }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        lg[st] = part + R.b3;
    }
}

__device__ __forceinline__ float pick4(const float (&v)[4], int i)
{
    return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}

// ---------------------------------------------------------------- kernels

// Logits of n samples X[n][48] (FP32 features), 256 samples per block.
__global__ __launch_bounds__(256) void mlp_infer_kernel(const float *__restrict__ th,
                                                        const float *__restrict__ X, int n,
                                                        float *__restrict__ logit)
{
    __shared__ short xs[256 * XS];
    const int tid = threadIdx.x;
    const long base = (long)blockIdx.x * 256;
    for (int e = tid; e < 256 * NIN; e += 256) {
        const int m = e / NIN, k = e - m * NIN;
        const long g = base + m;
        xs[m * XS + k] = g < n ? f2bf(X[g * NIN + k]) : (short)0;
    }
    __syncthreads();
    MlpRegs R;
    load_mlp(th, R);
    const int w = tid >> 6, l = tid & 63;
    float lg[4];
    mlp_wave(xs + w * 64 * XS, R, lg, nullptr, nullptr);
    const long g = base + tid;
    if (g < n) logit[g] = pick4(lg, l >> 4);
}

// Gradient of the mean binary cross-entropy over n samples: per block of
// 128 samples, the forward pass on MFMA, then the backward pass in FP32:
// per-sample deltas, then every parameter's sum over the block's samples.
// part[b][0..NPARAM-1] = gradient sums, part[b][NPARAM] = loss sum.
__global__ __launch_bounds__(128) void mlp_grad_kernel(const float *__restrict__ th,
                                                       const float *__restrict__ X,
                                                       const float *__restrict__ t, int n,
                                                       float invn, float *__restrict__ part)
{
    __shared__ short xs[128 * XS];
    __shared__ float a1s[128 * NH], a2s[128 * NH], d1s[128 * NH], d2s[128 * NH];
    __shared__ float gs[128], ls[128];
    const int tid = threadIdx.x;
    const long base = (long)blockIdx.x * 128;
    for (int e = tid; e < 128 * NIN; e += 128) {
        const int m = e / NIN, k = e - m * NIN;
        const long g = base + m;
        xs[m * XS + k] = g < n ? f2bf(X[g * NIN + k]) : (short)0;
    }
    __syncthreads();
    MlpRegs R;
    load_mlp(th, R);
    const int w = tid >> 6, l = tid & 63;
    float lg[4];
    mlp_wave(xs + w * 64 * XS, R, lg, a1s + w * 64 * NH, a2s + w * 64 * NH);
    const float z = pick4(lg, l >> 4);
    __syncthreads();
    const int m = tid;
    const long gi = base + m;
    float g = 0.f, lo = 0.f;
    if (gi < n) {
        const float tt = t[gi];
        const float y = 1.0f / (1.0f + expf(-z));
        g = (y - tt) * invn;
        lo = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - tt * z;
    }
    gs[m] = g;
    ls[m] = lo;
    for (int o = 0; o < NH; ++o) d2s[m * NH + o] = a2s[m * NH + o] > 0.f ? th[OW3 + o] * g : 0.f;
    for (int j = 0; j < NH; ++j) {
        float s = 0.f;
        for (int o = 0; o < NH; ++o) s += th[OW2 + o * NH + j] * d2s[m * NH + o];
        d1s[m * NH + j] = a1s[m * NH + j] > 0.f ? s : 0.f;
    }
    __syncthreads();
    float *pb = part + (long)blockIdx.x * (NPARAM + 1);
    for (int p = tid; p < NPARAM; p += 128) {
        float acc = 0.f;
        if (p < OB1) {
            const int o = p / NIN, k = p - o * NIN;
            for (int s = 0; s < 128; ++s) acc += d1s[s * NH + o] * bf2f(xs[s * XS + k]);
        } else if (p < OW2) {
            const int o = p - OB1;
            for (int s = 0; s < 128; ++s) acc += d1s[s * NH + o];
        } else if (p < OB2) {
            const int o = (p - OW2) / NH, k = (p - OW2) - o * NH;
            for (int s = 0; s < 128; ++s) acc += d2s[s * NH + o] * fmaxf(a1s[s * NH + k], 0.f);
        } else if (p < OW3) {
            const int o = p - OB2;
            for (int s = 0; s < 128; ++s) acc += d2s[s * NH + o];
        } else if (p < OB3) {
            const int o = p - OW3;
            for (int s = 0; s < 128; ++s) acc += gs[s] * fmaxf(a2s[s * NH + o], 0.f);
        } else {
            for (int s = 0; s < 128; ++s) acc += gs[s];
        }
        pb[p] = acc;
    }
    if (tid == 0) {
        float s = 0.f;
        for (int i = 0; i < 128; ++i) s += ls[i];
        pb[NPARAM] = s;
    }
}

// Sum the per-block partials in block order (deterministic).
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *__restrict__ part, int nblk,
                                                         float invn, float *__restrict__ grad,
                                                         float *__restrict__ loss)
{
    for (int p = threadIdx.x; p <= NPARAM; p += 256) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part[(long)b * (NPARAM + 1) + p];
        if (p < NPARAM) grad[p] = s;
        else if (loss) *loss = s * invn;
    }
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ th, float *__restrict__ mo,
                                                       float *__restrict__ ve,
                                                       const float *__restrict__ grad, float lr,
                                                       float b1, float b2, float eps, float c1,
                                                       float c2)
{
    for (int p = threadIdx.x + blockIdx.x * 256; p < NPARAM; p += 256 * gridDim.x) {
        const float g = grad[p];
        const float m = b1 * mo[p] + (1.f - b1) * g;
        const float v = b2 * ve[p] + (1.f - b2) * g * g;
        mo[p] = m;
        ve[p] = v;
        th[p] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
    }
}

// Relative excess of the full characteristic flux ff over the linear flux
// fl at one interface (both sweep-frame, rho, m_n, m_t1, m_t2, B_t1, B_t2,
// E): max over components of |ff - fl| / S, with a the largest |v_n| + c_f
// on the stencil and the scales S = a max rho (mass), a max(|m| + rho a)
// (momenta), a max(|B| + sqrt(rho) a) (fields), a max E (energy).
template <typename T>
__device__ T flux_excess(const T *__restrict__ sq, int qs, int off, int cstr, const T (&ff)[7],
                         const T (&fl)[7])
{
#define QE(q, j) sq[(q) * qs + off + (j) * cstr]
    T a = T(0);
    for (int j = 0; j < 6; ++j) a = fmax(a, fabs(QE(1, j) * QE(9, j)) + QE(10, j));
    T sr = T(0), sm = T(0), sb = T(0), se = T(0);
    for (int j = 0; j < 6; ++j) {
        const T r = QE(0, j);
        const T m = sqrt(QE(1, j) * QE(1, j) + QE(2, j) * QE(2, j) + QE(3, j) * QE(3, j));
        const T b = sqrt(QE(4, j) * QE(4, j) + QE(5, j) * QE(5, j) + QE(6, j) * QE(6, j));
        sr = fmax(sr, r);
        sm = fmax(sm, m + r * a);
        sb = fmax(sb, b + sqrt(r) * a);
        se = fmax(se, QE(7, j));
    }
#undef QE
    const T sc[7] = { sr, sm, sm, sm, sb, sb, se };
    T ex = T(0);
    for (int c = 0; c < 7; ++c) ex = fmax(ex, fabs(ff[c] - fl[c]) / (a * sc[c]));
    return ex;
}

// Training data: features, weight deviation and flux excess of n sampled
// interfaces where[s] = (dir, i, j, k) with i, j, k the face index along dir
// and interior cell indices on the other axes.  One thread per sample, its
// six cells staged in LDS.
template <typename T>
__global__ __launch_bounds__(64) void router_sample_kernel(const T *__restrict__ u, Geom G,
                                                           Phys P, const int32_t *__restrict__ where,
                                                           int n, float *__restrict__ X,
                                                           float *__restrict__ dev_out,
                                                           float *__restrict__ ex_out)
{
    __shared__ T sq[sw::NQ * 64 * 6];
    const int t = threadIdx.x;
    const long s = (long)blockIdx.x * 64 + t;
    bool ok = s < n;
    int dir = 0, pos[3] = { 0, 0, 0 };
    if (ok) {
        dir = where[4 * s];
        pos[0] = where[4 * s + 1];
        pos[1] = where[4 * s + 2];
        pos[2] = where[4 * s + 3];
        // only interfaces of the box: face index 0..n along an active dir,
        // interior cells on the other axes; anything else reads as NaN
        ok = dir >= 0 && dir < 3 && G.act[dir];
        for (int a = 0; a < 3 && ok; ++a)
            ok = pos[a] >= 0 && pos[a] <= G.n[a] - (a == dir ? 0 : 1);
        if (!ok) {
            for (int k = 0; k < 48; ++k) X[s * 48 + k] = __builtin_nanf("");
            dev_out[s] = ex_out[s] = __builtin_nanf("");
        }
    }
    if (ok) {
        const int t1 = (dir + 1) % 3, t2 = (dir + 2) % 3;
        const int cm[8] = { 0, 1 + dir, 1 + t1, 1 + t2, 4 + dir, 4 + t1, 4 + t2, 7 };
        for (int j = 0; j < 6; ++j) {
            int c[3] = { pos[0], pos[1], pos[2] };
            c[dir] = pos[dir] - 3 + j;
            const long id = G.base + c[0] * G.s[0] + c[1] * G.s[1] + (long)c[2] * G.s[2];
            sw::stage_cell(u, id, G.sv, cm, P.gamma, sq + t * 6 + j, 64 * 6);
        }
    }
    __syncthreads();
    if (!ok) return;
    float x[48];
    sw::router_features<T>(sq, 64 * 6, t * 6, 1, x);
    for (int k = 0; k < 48; ++k) X[s * 48 + k] = x[k];
    T ff[7], fl[7], dv = T(0);
    sw::face_flux<T, true>(sq, 64 * 6, t * 6, 1, P.gamma, P.igm1, (T)P.eps, ff, &dv);
    sw::linear_flux<T>(sq, 64 * 6, t * 6, 1, fl);
    dev_out[s] = (float)dv;
    ex_out[s] = (float)flux_excess<T>(sq, 64 * 6, t * 6, 1, ff, fl);
}

// Learned sweep (FP32 state): one tile of 256 interfaces as in the plain
// sweep (FT = 4); features -> MLP on MFMA -> routing; the block compacts
// its troubled and smooth interfaces into two lists so that full
// characteristic WENO and the linear flux each run on packed waves.
template <int DIR>
__global__ __launch_bounds__(256) void learned_sweep_kernel(const float *__restrict__ u,
                                                            float *__restrict__ flux, Geom G,
                                                            FaceBox F, Phys P,
                                                            const float *__restrict__ th,
                                                            float thr, int force,
                                                            int32_t *__restrict__ nsmooth)
{
    constexpr int FT = 4;
    constexpr int NC = sw::tile_cells<DIR, FT>();
    __shared__ float sq[sw::NQ * NC];
    __shared__ short xs[256 * XS];
    __shared__ unsigned short tl[256], sl[256];
    __shared__ int wcnt[8];
    constexpr int N = DIR;
    const int cm[8] = { 0, 1 + N, 1 + (N + 1) % 3, 1 + (N + 2) % 3, 4 + N, 4 + (N + 1) % 3,
                        4 + (N + 2) % 3, 7 };
    const int lane = threadIdx.x, w = threadIdx.y, tid = lane + 64 * w;
    const int ta = blockIdx.x, tb = blockIdx.y;
    const int nlast = G.n[N] + 2;
    // --- stage the tile (as sw::sweep_tile)
    if constexpr (DIR == 0) {
        const int nrows = F.cnt[1] * F.cnt[2];
        for (int c = tid; c < sw::ROWS * sw::NCX; c += 256) {
            int rr = c / sw::NCX, xi = c - rr * sw::NCX;
            int row = ta * sw::ROWS + rr, x = tb * sw::TILE - 3 + xi;
            if (row < nrows && x <= nlast) {
                int j = F.lo[1] + row % F.cnt[1], k = F.lo[2] + row / F.cnt[1];
                long id = G.base + x * G.s[0] + j * G.s[1] + k * G.s[2];
                sw::stage_cell(u, id, G.sv, cm, P.gamma, sq + c, NC);
            }
        }
    } else {
        constexpr int A = 0, B = (DIR == 1) ? 2 : 1;
        const int npos = F.cnt[A] * F.cnt[B];
        const int p = ta * 64 + lane;
        const int ca = F.lo[A] + p % F.cnt[A], cb = F.lo[B] + p / F.cnt[A];
        for (int rr = w; rr < FT + 5; rr += 4) {
            int y = tb * FT - 3 + rr;
            if (p < npos && y <= nlast) {
                long id = G.base + ca * G.s[A] + cb * G.s[B] + (long)y * G.s[N];
                sw::stage_cell(u, id, G.sv, cm, P.gamma, sq + rr * 64 + lane, NC);
            }
        }
    }
    __syncthreads();
    // --- interface t = 64*w + lane of the tile: position, activity, LDS offset
    auto where = [&](int t, int (&pos)[3], int &off, int &cstr) -> bool {
        const int ln = t & 63, ww = t >> 6;
        if constexpr (DIR == 0) {
            const int nrows = F.cnt[1] * F.cnt[2];
            const int row = ta * sw::ROWS + ww;
            pos[0] = tb * sw::TILE + ln;
            pos[1] = F.lo[1] + row % F.cnt[1];
            pos[2] = F.lo[2] + row / F.cnt[1];
            off = ww * sw::NCX + ln;
            cstr = 1;
            return row < nrows && pos[0] < F.cnt[0];
        } else {
            constexpr int A = 0, B = (DIR == 1) ? 2 : 1;
            const int npos = F.cnt[A] * F.cnt[B];
            const int p = ta * 64 + ln;
            pos[A] = F.lo[A] + p % F.cnt[A];
            pos[B] = F.lo[B] + p / F.cnt[A];
            pos[N] = tb * FT + ww;
            off = ww * 64 + ln;
            cstr = 64;
            return p < npos && pos[N] < F.cnt[N];
        }
    };
    int pos[3], off, cstr;
    const bool act = where(tid, pos, off, cstr);
    // --- features and the MLP
    {
        float x[48];
        if (act) sw::router_features<float>(sq, NC, off, cstr, x);
#pragma unroll
        for (int k = 0; k < 48; ++k) xs[tid * XS + k] = act ? f2bf(x[k]) : (short)0;
    }
    __syncthreads();
    bool troubled;
    if (force != 0) {
        troubled = force > 0;                 // routing switched off: all full / all linear
    } else {
        MlpRegs R;
        load_mlp(th, R);
        float lg[4];
        mlp_wave(xs + w * 64 * XS, R, lg, nullptr, nullptr);
        troubled = !(pick4(lg, lane >> 4) <= thr);      // NaN features count as troubled
    }
    // --- compaction: troubled list tl, smooth list sl (block order)
    const unsigned long long bt = __ballot(act && troubled), bs = __ballot(act && !troubled);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) { wcnt[w] = __popcll(bt); wcnt[4 + w] = __popcll(bs); }
    __syncthreads();
    int ot = 0, os = 0;
    for (int i = 0; i < w; ++i) { ot += wcnt[i]; os += wcnt[4 + i]; }
    const int ntr = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    const int nsm = wcnt[4] + wcnt[5] + wcnt[6] + wcnt[7];
    if (act && troubled) tl[ot + __popcll(bt & below)] = (unsigned short)tid;
    if (act && !troubled) sl[os + __popcll(bs & below)] = (unsigned short)tid;
    __syncthreads();
    if (tid == 0 && nsmooth) nsmooth[(long)blockIdx.y * gridDim.x + blockIdx.x] = nsm;
    // --- fluxes on packed waves
    for (int k = tid; k < ntr; k += 256) {
        int p2[3], o2, c2;
        where(tl[k], p2, o2, c2);
        float out[7];
        sw::face_flux<float>(sq, NC, o2, c2, P.gamma, P.igm1, (float)P.eps, out);
        sw::store_face<N, float>(flux, F, p2, out);
    }
    for (int k = tid; k < nsm; k += 256) {
        int p2[3], o2, c2;
        where(sl[k], p2, o2, c2);
        float out[7];
        sw::linear_flux<float>(sq, NC, o2, c2, out);
        sw::store_face<N, float>(flux, F, p2, out);
    }
}

}  // namespace rt

// ---------------------------------------------------------------- launchers

hipError_t launch_mlp_infer(const float *th, const float *X, int n, float *logit, hipStream_t st)
{
    hipLaunchKernelGGL(rt::mlp_infer_kernel, dim3((n + 255) / 256), dim3(256), 0, st, th, X, n, logit);
    return hipGetLastError();
}

int mlp_grad_blocks(int n) { return (n + 127) / 128; }

hipError_t launch_mlp_grad(const float *th, const float *X, const float *t, int n, float *part,
                           float *grad, float *loss, hipStream_t st)
{
    const int nb = mlp_grad_blocks(n);
    const float invn = 1.0f / (float)n;
    hipLaunchKernelGGL(rt::mlp_grad_kernel, dim3(nb), dim3(128), 0, st, th, X, t, n, invn, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rt::mlp_reduce_kernel, dim3(1), dim3(256), 0, st, part, nb, invn, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *th, float *m, float *v, const float *grad, int step, float lr,
                           float b1, float b2, float eps, hipStream_t st)
{
    const float c1 = 1.0f / (1.0f - powf(b1, (float)step));
    const float c2 = 1.0f / (1.0f - powf(b2, (float)step));
    hipLaunchKernelGGL(rt::mlp_adam_kernel, dim3(11), dim3(256), 0, st, th, m, v, grad, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_router_sample(const T *u, const Geom &G, const Phys &P, const int32_t *where,
                                int n, float *X, float *dev, float *ex, hipStream_t st)
{
    hipLaunchKernelGGL((rt::router_sample_kernel<T>), dim3((n + 63) / 64), dim3(64), 0, st, u, G, P,
                       where, n, X, dev, ex);
    return hipGetLastError();
}
template hipError_t launch_router_sample<double>(const double *, const Geom &, const Phys &,
                                                 const int32_t *, int, float *, float *, float *,
                                                 hipStream_t);
template hipError_t launch_router_sample<float>(const float *, const Geom &, const Phys &,
                                                const int32_t *, int, float *, float *, float *,
                                                hipStream_t);

long learned_sweep_blocks(int dir, const FaceBox &F)
{
    long na, nb;
    if (dir == 0) sw::sweep_tiles<0, 4>(F, na, nb);
    else if (dir == 1) sw::sweep_tiles<1, 4>(F, na, nb);
    else sw::sweep_tiles<2, 4>(F, na, nb);
    return na * nb;
}

hipError_t launch_learned_sweep(int dir, const float *u, float *flux, const Geom &G, const FaceBox &F,
                                const Phys &P, const float *th, float thr, int force,
                                int32_t *nsmooth, hipStream_t st)
{
    long na, nb;
    dim3 blk(64, 4);
    switch (dir) {
    case 0:
        sw::sweep_tiles<0, 4>(F, na, nb);
        hipLaunchKernelGGL(rt::learned_sweep_kernel<0>, dim3((unsigned)na, (unsigned)nb), blk, 0, st, u,
                           flux, G, F, P, th, thr, force, nsmooth);
        break;
    case 1:
        sw::sweep_tiles<1, 4>(F, na, nb);
        hipLaunchKernelGGL(rt::learned_sweep_kernel<1>, dim3((unsigned)na, (unsigned)nb), blk, 0, st, u,
                           flux, G, F, P, th, thr, force, nsmooth);
        break;
    default:
        sw::sweep_tiles<2, 4>(F, na, nb);
        hipLaunchKernelGGL(rt::learned_sweep_kernel<2>, dim3((unsigned)na, (unsigned)nb), blk, 0, st, u,
                           flux, G, F, P, th, thr, force, nsmooth);
        break;
    }
    return hipGetLastError();
}

}  // namespace ww
