// ww_router.hip -- the learned troubled-interface router.
//
// An MLP 48 -> 32 -> 32 -> 1 (ReLU, sigmoid) reads log-scaled difference
// magnitudes of the six-cell stencil of an interface and predicts whether
// the full characteristic WENO flux (arXiv:1808.10633 Sec. 2.1) is needed
// there, i.e. whether it departs from the linear fifth-order component-wise
// flux by more than a set fraction of the local flux scale (the flux
// excess).  Interfaces called smooth take the linear flux instead.
//
// Matrix products run on MFMA (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32
// accumulation).  Layers are computed transposed, Z^T = W X^T, so that the
// output registers of one layer (lane l holds rows 4(l/16)+i, column l%16 of
// a 16x16 tile) are exactly the B operand of the next layer: no shuffles.
// Parameters are one FP32 vector of 2657 values: W1 (32x48, [out][in]), b1,
// W2 (32x32), b2, w3 (32), b3.  Training kernels convert them per block; the
// routed sweep reads a copy packed once in the per-lane operand order.
#include "ww_router.h"
#include "ww_sweep_dev.h"

namespace ww {
namespace rt {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int YZ_PW = 32;         // positions per y/z tile of the routed sweep (8 faces each)
constexpr int QREG = 64;          // troubled-queue regions (atomic counters)
static_assert(QREG == ROUTED_QUEUE_REGIONS, "queue regions");
constexpr int OW1 = 0, OB1 = 1536, OW2 = 1568, OB2 = 2592, OW3 = 2624, OB3 = 2656;
constexpr int XS = 52;     // LDS row stride (BF16 elements) of the feature matrix

__device__ __forceinline__ short f2bf(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);      // round to nearest even
    return (short)(u >> 16);
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

// Parameters packed for the routed sweep: [10][64] BF16 operand fragments
// (a1 by (ot, kt), then a2 by (ot, kt)) followed by [25][64] floats (b1, b2,
// w3 by (ot, i), then b3), item-major so that a wave reads every item with
// one coalesced load and converts nothing.
__global__ __launch_bounds__(64) void pack_mlp_kernel(const float *__restrict__ th, char *__restrict__ pk)
{
    const int l = threadIdx.x;
    MlpRegs R;
    load_mlp(th, R);
    bf4 *pa = (bf4 *)pk;
    float *pf = (float *)(pk + 10 * 64 * 8);
    int t = 0;
    for (int ot = 0; ot < 2; ++ot)
        for (int kt = 0; kt < 3; ++kt) pa[64 * t++ + l] = R.a1[ot][kt];
    for (int ot = 0; ot < 2; ++ot)
        for (int kt = 0; kt < 2; ++kt) pa[64 * t++ + l] = R.a2[ot][kt];
    t = 0;
    for (int ot = 0; ot < 2; ++ot)
        for (int i = 0; i < 4; ++i) {
            pf[64 * (t + 0) + l] = R.b1[ot][i];
            pf[64 * (t + 8) + l] = R.b2[ot][i];
            pf[64 * (t + 16) + l] = R.w3[ot][i];
            ++t;
        }
    pf[64 * 24 + l] = R.b3;
}

__device__ __forceinline__ void load_mlp_packed(const char *__restrict__ pk, MlpRegs &R)
{
    const int l = threadIdx.x & 63;
    const bf4 *pa = (const bf4 *)pk;
    const float *pf = (const float *)(pk + 10 * 64 * 8);
    int t = 0;
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
        for (int kt = 0; kt < 3; ++kt) R.a1[ot][kt] = pa[64 * t++ + l];
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) R.a2[ot][kt] = pa[64 * t++ + l];
    t = 0;
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            R.b1[ot][i] = pf[64 * (t + 0) + l];
            R.b2[ot][i] = pf[64 * (t + 8) + l];
            R.w3[ot][i] = pf[64 * (t + 16) + l];
            ++t;
        }
    R.b3 = pf[64 * 24 + l];
}

// Four floats as four BF16 (round to nearest even, hardware conversion).
__device__ __forceinline__ bf4 pack_bf4(float a, float b, float c, float d)
{
    typedef __bf16 h4 __attribute__((ext_vector_type(4)));
    const h4 v = { (__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d };
    return __builtin_bit_cast(bf4, v);
}

// Forward pass of 16 samples, rows g[m*XS + k] (BF16), m = 0..15; returns
// the logit of sample l%16 (in every lane).
__device__ __forceinline__ float mlp_group(const short *g, const MlpRegs &R)
{
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    f4 z1[2] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
#pragma unroll
    for (int kt = 0; kt < 3; ++kt) {
        const bf4 bx = *(const bf4 *)(g + r * XS + 16 * kt + 4 * q);
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
            part += R.w3[ot][i] * fmaxf(a, 0.f);
        }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    return part + R.b3;
}

// Forward pass of the 64 samples of this wave, rows xs[m*XS + k] (BF16),
// m = 0..63.  lg[st] receives the logit of sample 16*st + l%16.
__device__ __forceinline__ void mlp_wave(const short *xs, const MlpRegs &R, float (&lg)[4])
{
#pragma unroll
    for (int st = 0; st < 4; ++st) lg[st] = mlp_group(xs + 16 * st * XS, R);
}

__device__ __forceinline__ float pick4(const float (&v)[4], int i)
{
    return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}

// ---------------------------------------------------------------- stencil

// Stencil scales shared by the features and the flux excess: a = the
// largest |v_n| + c_f on the stencil; S = max rho (mass), max(|m|_1 + rho a)
// (momenta), max |B|_1 + sqrt(max rho) a (fields), max E (energy), returned
// as reciprocals is[4].  (|.|_1: sum of the absolute components.)
template <typename T>
__device__ __forceinline__ void stencil_scales(const T *__restrict__ sq, int qs, int off, int cstr,
                                               T &a, T (&is)[4])
{
#define QS(q, j) sq[(q) * qs + off + (j) * cstr]
    a = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) a = fmax(a, fabs(QS(1, j)) * QS(9, j) + QS(10, j));
    T sr = T(0), sm = T(0), sb = T(0), se = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const T r = QS(0, j);
        sr = fmax(sr, r);
        sm = fmax(sm, fabs(QS(1, j)) + fabs(QS(2, j)) + fabs(QS(3, j)) + r * a);
        sb = fmax(sb, fabs(QS(4, j)) + fabs(QS(5, j)) + fabs(QS(6, j)));
        se = fmax(se, QS(7, j));
    }
#undef QS
    sb += sqrt(sr) * a;
    is[0] = sw::frcp(sr);
    is[1] = sw::frcp(sm);
    is[2] = sw::frcp(sb);
    is[3] = sw::frcp(se);
}

// log2 by Mitchell's approximation (exponent plus the mantissa fraction,
// read off the bit pattern), exact at powers of two, error below 0.087.
__device__ __forceinline__ float log2m(float y)
{
    return (float)__float_as_int(y) * 1.1920928955078125e-07f - 127.0f;
}

// Router features of one interface from its six staged cells (i-2..i+3),
// six per sweep-frame conserved variable v, stored x[v*6 + j], each
// L(y) = 1 + log2m(y / S_v + 1e-8) log10(2) / 4 of
//   j = 0     the largest first difference on the stencil,
//   j = 1     the jump across the interface |q_3 - q_2|,
//   j = 2..4  the largest second, third and fourth difference,
//   j = 5     the fifth difference (absolute values throughout).
// On smooth data the m-th difference falls like (kh)^m, so smoothness and
// amplitude are both differences of O(1) features, which BF16 carries.
template <typename T>
__device__ __forceinline__ void router_features(const T *__restrict__ sq, int qs, int off, int cstr,
                                                float (&x)[48])
{
#define QF(q, j) sq[(q) * qs + off + (j) * cstr]
    T a, is[4];
    stencil_scales<T>(sq, qs, off, cstr, a, is);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const T iv = is[v == 0 ? 0 : v < 4 ? 1 : v < 7 ? 2 : 3];
        T d[6], y[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) d[j] = QF(v, j);
        y[1] = fabs(d[3] - d[2]);
#pragma unroll
        for (int m = 1; m <= 5; ++m) {           // d <- its next difference
            T mx = T(0);
#pragma unroll
            for (int j = 0; j + m < 6; ++j) { d[j] = d[j + 1] - d[j]; mx = fmax(mx, fabs(d[j])); }
            y[m == 1 ? 0 : m] = mx;
        }
#pragma unroll
        for (int j = 0; j < 6; ++j)
            x[v * 6 + j] = 1.0f + 0.0752574989f * log2m((float)(y[j] * iv + T(1e-8)));
    }
#undef QF
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
    mlp_wave(xs + w * 64 * XS, R, lg);
    const long g = base + tid;
    if (g < n) logit[g] = pick4(lg, l >> 4);
}

// Gradient of the mean binary cross-entropy over n samples, 128 samples per
// block (two waves of 64), every product on MFMA (BF16 operands, FP32
// accumulation):
//   forward   Z1^T = W1 X^T, Z2^T = W2 H1^T (as in inference), logit in FP32;
//   deltas    g = (sigmoid(logit) - t) / n, D2 = w3 g [z2 > 0] (per sample),
//             D1^T = W2^T D2^T, masked by [z1 > 0]: the C-layout registers of
//             D2^T are the B operand of this product (no shuffles), and the
//             result lands in the layout of Z1^T, whose mask sits in the same
//             registers;
//   weights   dW1 | db1 = D1^T [X | 1], dW2 | db2 = D2^T [H1 | 1]: products
//             over the block's 128 samples (K = samples), with a row of ones
//             appended to the sample-contiguous LDS copies of X and H1 so the
//             bias gradients come out of the same MFMAs; dw3 = g^T H2 and
//             db3 = sum g are reduced across lanes in FP32.
// Rounding points (mirrored by the element-wise test): X, W1, W2, H1 = relu(z1),
// D2 and the masked D1 are rounded to BF16; z1, z2, H2, the logit, g and every
// sum are FP32.  part[b][0..NPARAM-1] = the block's gradient sums,
// part[b][NPARAM] = its loss sum.
constexpr int TS = 136;          // LDS row stride (BF16 elements) of the sample-contiguous copies

__global__ __launch_bounds__(128) void mlp_grad_kernel(const float *__restrict__ th,
                                                       const float *__restrict__ X,
                                                       const float *__restrict__ t, int n,
                                                       float invn, float *__restrict__ part)
{
    __shared__ short xs[128 * XS];       // [sample][feature]: forward B operand
    __shared__ short xT[64 * TS];        // [feature | ones | zeros][sample]
    __shared__ short h1T[48 * TS];       // [hidden 1 | ones | zeros][sample]
    __shared__ short d1T[32 * TS], d2T[32 * TS];
    __shared__ float red[2][NH + 2];
    const int tid = threadIdx.x;
    const long base = (long)blockIdx.x * 128;
    for (int e = tid; e < 128 * NIN; e += 128) {
        const int m = e / NIN, k = e - m * NIN;
        const long g = base + m;
        const short v = g < n ? f2bf(X[g * NIN + k]) : (short)0;
        xs[m * XS + k] = v;
        xT[k * TS + m] = v;
    }
    const short one = f2bf(1.0f);
    for (int e = tid; e < 16 * 128; e += 128) {
        const int rr = e >> 7, m = e & 127;
        xT[(NIN + rr) * TS + m] = rr == 0 ? one : (short)0;
        h1T[(NH + rr) * TS + m] = rr == 0 ? one : (short)0;
    }
    __syncthreads();
    MlpRegs R;
    load_mlp(th, R);
    const int w = tid >> 6, l = tid & 63, r = l & 15, q = l >> 4;
    // W2^T in A-operand order: tile (jt, kt), lane holds W2^T[16jt + r][16kt + 4q + i]
    bf4 a2t[2][2];
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) a2t[jt][kt][i] = f2bf(th[OW2 + (16 * kt + 4 * q + i) * NH + 16 * jt + r]);
    float gw3[2][4] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
    float gb3 = 0.f, gl = 0.f;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int col = 64 * w + 16 * st + r;          // this lane's sample within the block
        const short *gx = xs + (64 * w + 16 * st) * XS;
        f4 z1[2] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
#pragma unroll
        for (int kt = 0; kt < 3; ++kt) {
            const bf4 bx = *(const bf4 *)(gx + r * XS + 16 * kt + 4 * q);
#pragma unroll
            for (int ot = 0; ot < 2; ++ot)
                z1[ot] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a1[ot][kt], bx, z1[ot], 0, 0, 0);
        }
        bf4 h1[2];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z1[ot][i] += R.b1[ot][i];
                h1[ot][i] = f2bf(fmaxf(z1[ot][i], 0.f));
                h1T[(16 * ot + 4 * q + i) * TS + col] = h1[ot][i];
            }
        f4 z2[2] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int ot = 0; ot < 2; ++ot)
                z2[ot] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a2[ot][kt], h1[kt], z2[ot], 0, 0, 0);
        float zl = 0.f;
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z2[ot][i] += R.b2[ot][i];
                zl += R.w3[ot][i] * fmaxf(z2[ot][i], 0.f);
            }
        zl += __shfl_xor(zl, 16);
        zl += __shfl_xor(zl, 32);
        const float z = zl + R.b3;                     // logit of sample `col` (every q)
        const long gi = base + col;
        float g = 0.f, lo = 0.f;
        if (gi < n) {
            const float tt = t[gi];
            g = (1.0f / (1.0f + expf(-z)) - tt) * invn;
            lo = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - tt * z;
        }
        if (q == 0) { gb3 += g; gl += lo; }
        bf4 d2[2];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float h2 = fmaxf(z2[ot][i], 0.f);
                gw3[ot][i] += g * h2;
                d2[ot][i] = f2bf(z2[ot][i] > 0.f ? R.w3[ot][i] * g : 0.f);
                d2T[(16 * ot + 4 * q + i) * TS + col] = d2[ot][i];
            }
        f4 d1[2] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int jt = 0; jt < 2; ++jt)
                d1[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2t[jt][kt], d2[kt], d1[jt], 0, 0, 0);
#pragma unroll
        for (int jt = 0; jt < 2; ++jt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                d1T[(16 * jt + 4 * q + i) * TS + col] = f2bf(z1[jt][i] > 0.f ? d1[jt][i] : 0.f);
    }
    // dw3, db3 and the loss: sums over the 16 lanes of a row group, then the two waves
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) {
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int i = 0; i < 4; ++i) gw3[ot][i] += __shfl_xor(gw3[ot][i], m);
        gb3 += __shfl_xor(gb3, m);
        gl += __shfl_xor(gl, m);
    }
    if (r == 0) {
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[w][16 * ot + 4 * q + i] = gw3[ot][i];
        if (q == 0) { red[w][NH] = gb3; red[w][NH + 1] = gl; }
    }
    __syncthreads();
    float *pb = part + (long)blockIdx.x * (NPARAM + 1);
    if (tid < NH) pb[OW3 + tid] = red[0][tid] + red[1][tid];
    if (tid == NH) pb[OB3] = red[0][NH] + red[1][NH];
    if (tid == NH + 1) pb[NPARAM] = red[0][NH + 1] + red[1][NH + 1];
    // weight gradients over the 128 samples: wave w takes output rows 16w..16w+15
    f4 g1[4] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f },
                 { 0.f, 0.f, 0.f, 0.f } };
    f4 g2[3] = { { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f }, { 0.f, 0.f, 0.f, 0.f } };
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        const int s0 = 16 * ks + 4 * q;
        const bf4 a1 = *(const bf4 *)(d1T + (16 * w + r) * TS + s0);
        const bf4 a2 = *(const bf4 *)(d2T + (16 * w + r) * TS + s0);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            g1[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, *(const bf4 *)(xT + (16 * nt + r) * TS + s0),
                                                               g1[nt], 0, 0, 0);
#pragma unroll
        for (int nt = 0; nt < 3; ++nt)
            g2[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, *(const bf4 *)(h1T + (16 * nt + r) * TS + s0),
                                                               g2[nt], 0, 0, 0);
    }
    // lane holds D[row 16w + 4q + i][column 16nt + r]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = 16 * w + 4 * q + i;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int k = 16 * nt + r;
            if (k < NIN) pb[OW1 + o * NIN + k] = g1[nt][i];
            else if (k == NIN) pb[OB1 + o] = g1[nt][i];
        }
#pragma unroll
        for (int nt = 0; nt < 3; ++nt) {
            const int j = 16 * nt + r;
            if (j < NH) pb[OW2 + o * NH + j] = g2[nt][i];
            else if (j == NH) pb[OB2 + o] = g2[nt][i];
        }
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
// E): max over components of |ff - fl| / (a S) with the stencil scales.
template <typename T>
__device__ T flux_excess(const T *__restrict__ sq, int qs, int off, int cstr, const T (&ff)[7],
                         const T (&fl)[7])
{
    T a, is[4];
    stencil_scales<T>(sq, qs, off, cstr, a, is);
    const int g[7] = { 0, 1, 1, 1, 2, 2, 3 };
    T ex = T(0);
#pragma unroll
    for (int c = 0; c < 7; ++c) ex = fmax(ex, fabs(ff[c] - fl[c]) * is[g[c]]);
    return ex / a;
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
    router_features<T>(sq, 64 * 6, t * 6, 1, x);
    for (int k = 0; k < 48; ++k) X[s * 48 + k] = x[k];
    T ff[7], fl[7], dv = T(0);
    sw::face_flux<T, true>(sq, 64 * 6, t * 6, 1, P.gamma, P.igm1, (T)P.eps, ff, &dv);
    sw::linear_flux<T>(sq, 64 * 6, t * 6, 1, fl);
    dev_out[s] = (float)dv;
    ex_out[s] = (float)flux_excess<T>(sq, 64 * 6, t * 6, 1, ff, fl);
}

// Routed sweep (FP32 state): one tile of 256 interfaces, one per thread.
// Features -> MLP on MFMA -> the interfaces called smooth
// take the linear flux here; the troubled ones are appended to a queue that
// troubled_kernel serves with full characteristic WENO in packed waves, so a
// few troubled interfaces in a tile cost a few queue slots, not a wave.
// The queue is split into QREG regions (block b appends to region b % QREG,
// of capacity qcap entries) so that the one atomic reservation per block
// spreads over QREG counters instead of contending on one.
// force = -1: every interface smooth, the network not evaluated.  reuse:
// take the decisions stored in mask (one byte per face, 1 = troubled) by an
// earlier evaluation instead of evaluating the network; otherwise store them.
// Queue entries pack the face position (x+1, y+1, z+1) in 21 bits each.
// FUSED (x sweep, flattened 256-face tiles, after the y and z sweeps): the
// tile also applies the rho, m, E update (RK stage xf.c) to every cell whose
// two x faces lie in the tile and are both smooth, with their fluxes from
// LDS (the fused x sweep's tail); the other cells are left to
// xfix_queue_kernel and xfix_bound_kernel.
template <int DIR, bool FUSED = false>
__global__ __launch_bounds__(256) void routed_sweep_kernel(const float *__restrict__ u,
                                                           float *__restrict__ flux, Geom G,
                                                           FaceBox F, Phys P,
                                                           const char *__restrict__ pk,
                                                           float thr, int force,
                                                           int32_t *__restrict__ nsmooth,
                                                           unsigned long long *__restrict__ queue,
                                                           int32_t *__restrict__ qcount, long qcap,
                                                           unsigned char *__restrict__ mask, int reuse,
                                                           XFuse<float> xf)
{
    static_assert(!FUSED || DIR == 0, "the fused tail belongs to the x sweep");
    // tiles as the plain sweeps: x in flattened 256-face segments (rows of
    // XSEG_MIN faces or more) or 4 rows x 64 faces; y/z 32 positions x 8 faces
    constexpr int NC = DIR == 0 ? sw::XSEG_CELLS : sw::yz_cells<YZ_PW>();
    __shared__ float sq[sw::NQ * NC];
    __shared__ __align__(16) short xs[4 * 32 * XS];     // 32 feature rows per wave
    __shared__ int wcnt[4], wact[4];
    __shared__ long qbase;
    __shared__ float hx[FUSED ? 5 * 256 : 1];           // FUSED: rho, m, E fluxes of the tile's smooth faces
    __shared__ unsigned char tfl[FUSED ? 256 : 1];     // FUSED: 1 = no flux of this face in hx
    constexpr int N = DIR;
    const int lane = threadIdx.x, w = threadIdx.y, tid = lane + 64 * w;
    int pos[3], off, cstr;
    bool act;
    int nface = 0;
    sw::stage_begin();
    if constexpr (DIR == 0) {
        cstr = 1;
        if (FUSED || F.cnt[0] >= sw::XSEG_MIN) {
            const sw::XSeg X = sw::xseg_setup(F, blockIdx.x);
            sw::xseg_stage<float, false, true>(u, G, F, P, X, sq);
            __syncthreads();
            sw::stage_end();
            act = sw::xseg_face(F, X, tid, pos, off);
            nface = X.nface;
        } else {
            const int cm[8] = { 0, 1, 2, 3, 4, 5, 6, 7 };
            const int ta = blockIdx.x, tb = blockIdx.y, nlast = G.n[0] + 2;
            const int nrows = F.cnt[1] * F.cnt[2];
            for (int c = tid; c < sw::ROWS * sw::NCX; c += 256) {
                int rr = c / sw::NCX, xi = c - rr * sw::NCX;
                int row = ta * sw::ROWS + rr, x = tb * sw::TILE - 3 + xi;
                if (row < nrows && x <= nlast) {
                    int j = F.lo[1] + row % F.cnt[1], k = F.lo[2] + row / F.cnt[1];
                    long id = G.base + x * G.s[0] + j * G.s[1] + k * G.s[2];
                    sw::stage_cell<float, false, true>(u, id, G.sv, cm, P.gamma, sq + c, NC);
                }
            }
            __syncthreads();
            sw::stage_end();
            const int row = ta * sw::ROWS + w;
            pos[0] = tb * sw::TILE + lane;
            pos[1] = F.lo[1] + row % F.cnt[1];
            pos[2] = F.lo[2] + row / F.cnt[1];
            off = w * sw::NCX + lane;
            act = row < nrows && pos[0] < F.cnt[0];
        }
    } else {
        cstr = YZ_PW;
        sw::yz_stage<DIR, YZ_PW, float, true>(u, G, F, P, blockIdx.x, blockIdx.y, sq);
        __syncthreads();
        sw::stage_end();
        act = sw::yz_face<DIR, YZ_PW>(F, blockIdx.x, blockIdx.y, tid, pos, off);
    }
    // --- features and the MLP
    bool troubled = false;
    if (force == 0 && reuse) {
        troubled = act && mask[F.idx(pos[0], pos[1], pos[2])] != 0;
    } else if (force == 0) {
        bf4 xb[12];
        {
            float x[48];
            if (act) router_features<float>(sq, NC, off, cstr, x);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                xb[k] = act ? pack_bf4(x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]) : bf4{ 0, 0, 0, 0 };
        }
        MlpRegs R;
        load_mlp_packed(pk, R);
        short *g = xs + w * 32 * XS;
        float lg = 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // the 32 lanes of groups 2h, 2h+1 put their features in the wave's rows
            if ((lane >> 5) == h) {
                bf4 *row = (bf4 *)(g + (lane & 31) * XS);
#pragma unroll
                for (int k = 0; k < 12; ++k) row[k] = xb[k];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const float z0 = mlp_group(g, R);
            const float z1 = mlp_group(g + 16 * XS, R);
            if ((lane >> 4) == 2 * h) lg = z0;
            if ((lane >> 4) == 2 * h + 1) lg = z1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        troubled = !(lg <= thr);                // NaN features count as troubled
        if (act) mask[F.idx(pos[0], pos[1], pos[2])] = troubled ? 1 : 0;
    }
    // smooth interfaces: the linear flux (stored below)
    float lin[7];
    if (act && !troubled) sw::linear_flux<float>(sq, NC, off, cstr, lin);
    if constexpr (FUSED) {
        const bool have = act && !troubled;
        tfl[tid] = have ? 0 : 1;
        if (have) {
            hx[0 * 256 + tid] = lin[0];
            hx[1 * 256 + tid] = lin[1];
            hx[2 * 256 + tid] = lin[2];
            hx[3 * 256 + tid] = lin[3];
            hx[4 * 256 + tid] = lin[6];
        }
    }
    // --- troubled interfaces: one queue reservation per block
    const unsigned long long bt = __ballot(act && troubled), ba = __ballot(act);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) { wcnt[w] = __popcll(bt); wact[w] = __popcll(ba); }
    __syncthreads();
    const int ntr = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (tid == 0) {
        const int nact = wact[0] + wact[1] + wact[2] + wact[3];
        if (nsmooth) nsmooth[(long)blockIdx.y * gridDim.x + blockIdx.x] = nact - ntr;
        const long b = (long)blockIdx.y * gridDim.x + blockIdx.x;
        const int reg = (int)(b % QREG);
        qbase = ntr > 0 ? (long)reg * qcap + atomicAdd(qcount + reg, ntr) : 0;
    }
    __syncthreads();
    if (act && troubled) {
        long o = qbase;
        for (int i = 0; i < w; ++i) o += wcnt[i];
        o += __popcll(bt & below);
        queue[o] = (unsigned long long)(pos[0] + 1) | ((unsigned long long)(pos[1] + 1) << 21) |
                   ((unsigned long long)(pos[2] + 1) << 42);
    }
    if (act && !troubled) sw::store_face<N, float>(flux, F, pos, lin);
    if constexpr (FUSED) {
        // the cell between faces tid and tid + 1 (same row, interior), both
        // smooth; hx and tfl were published by the barrier above
        const int i = pos[0], j = pos[1], k = pos[2];
        const bool cell = act && tid + 1 < nface && i + 1 < F.cnt[0] && j >= 0 && j < G.n[1] && k >= 0 &&
                          k < G.n[2] && tfl[tid] == 0 && tfl[tid + 1] == 0;
        if (cell) {
            sw::FusedCell<float> fc;
            sw::fused_cell_load<float>(xf, G, i, j, k, fc);
            sw::fused_cell_store<float>(xf, G, hx, 256, tid, fc);
        }
    }
}

// The rho, m, E update of one cell left by the fused routed x sweep, its x
// fluxes read back from the flux buffer (every x face stored by then).
__device__ __forceinline__ void xfix_cell(const float *__restrict__ flux, const Geom &G, const FaceBox &F,
                                          const XFuse<float> &xf, int i, int j, int k)
{
    const int hs[5] = { 0, 1, 2, 3, 6 };
    float xl[5], xr[5];
    const long fl = F.idx(i, j, k), fr = F.idx(i + 1, j, k);
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        xl[h] = flux[hs[h] * F.sc + fl];
        xr[h] = flux[hs[h] * F.sc + fr];
    }
    sw::FusedCell<float> fc;
    sw::fused_cell_load<float>(xf, G, i, j, k, fc);
    sw::fused_cell_rk<float>(xf, G, xl, xr, fc);
}

// After the troubled pass: the cells next to the troubled x faces of queue
// region blockIdx.y.  Each such cell is taken once: the cell right of a
// troubled face by that face's entry, the cell left of it only if its own
// lower face is smooth (else that face's entry takes it).
__global__ __launch_bounds__(128) void xfix_queue_kernel(const float *__restrict__ flux, Geom G, FaceBox F,
                                                         XFuse<float> xf,
                                                         const unsigned long long *__restrict__ queue,
                                                         const int32_t *__restrict__ qcount, long qcap,
                                                         const unsigned char *__restrict__ mask)
{
    const long n = qcount[blockIdx.y];
    const unsigned long long *qr = queue + blockIdx.y * qcap;
    for (long e = (long)blockIdx.x * 128 + threadIdx.x; e < n; e += (long)gridDim.x * 128) {
        const unsigned long long q = qr[e];
        const int i = (int)(q & 0x1fffff) - 1, j = (int)((q >> 21) & 0x1fffff) - 1, k = (int)(q >> 42) - 1;
        if (j < 0 || j >= G.n[1] || k < 0 || k >= G.n[2]) continue;
        if (i < G.n[0]) xfix_cell(flux, G, F, xf, i, j, k);
        if (i > 0 && mask[F.idx(i - 1, j, k)] == 0) xfix_cell(flux, G, F, xf, i - 1, j, k);
    }
}

// The cells whose two x faces are smooth but lie in consecutive tiles (tile
// t ends with face 256 t + 255), one thread per tile boundary.  Decisions
// from mask (force -1: every face smooth).
__global__ __launch_bounds__(256) void xfix_bound_kernel(const float *__restrict__ flux, Geom G, FaceBox F,
                                                         XFuse<float> xf, const unsigned char *__restrict__ mask,
                                                         int force, long ntile)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t + 1 >= ntile) return;
    const int nf = F.cnt[0];
    const long g = 256 * t + 255, row = g / nf;
    const int i = (int)(g - row * nf);
    if (i + 1 >= nf) return;                                 // the row ends there: no cell
    const int j = F.lo[1] + (int)(row % F.cnt[1]), k = F.lo[2] + (int)(row / F.cnt[1]);
    if (j < 0 || j >= G.n[1] || k < 0 || k >= G.n[2]) return;
    if (force == 0 && (mask[F.idx(i, j, k)] != 0 || mask[F.idx(i + 1, j, k)] != 0)) return;
    xfix_cell(flux, G, F, xf, i, j, k);
}

// Full characteristic WENO at the queued troubled interfaces: each thread
// stages its own six cells and computes one flux; blockIdx.y is the queue
// region, whose length the routed sweep left in qcount[region], and the
// blocks of a region stride over it.
template <int DIR>
__global__ __launch_bounds__(128) void troubled_kernel(const float *__restrict__ u,
                                                       float *__restrict__ flux, Geom G, FaceBox F,
                                                       Phys P,
                                                       const unsigned long long *__restrict__ queue,
                                                       const int32_t *__restrict__ qcount, long qcap)
{
    __shared__ float sq[sw::NQ * 128 * 6];
    constexpr int N = DIR;
    const int cm[8] = { 0, 1 + N, 1 + (N + 1) % 3, 1 + (N + 2) % 3, 4 + N, 4 + (N + 1) % 3,
                        4 + (N + 2) % 3, 7 };
    const int t = threadIdx.x;
    const long n = qcount[blockIdx.y];
    const unsigned long long *qr = queue + blockIdx.y * qcap;
    for (long e = (long)blockIdx.x * 128 + t; e - t < n; e += (long)gridDim.x * 128) {
        if (e >= n) continue;
        const unsigned long long q = qr[e];
        int pos[3] = { (int)(q & 0x1fffff) - 1, (int)((q >> 21) & 0x1fffff) - 1, (int)(q >> 42) - 1 };
        for (int j = 0; j < 6; ++j) {
            int c[3] = { pos[0], pos[1], pos[2] };
            c[N] = pos[N] - 3 + j;
            const long id = G.base + c[0] * G.s[0] + c[1] * G.s[1] + (long)c[2] * G.s[2];
            sw::stage_cell(u, id, G.sv, cm, P.gamma, sq + t * 6 + j, 128 * 6);
        }
        float out[7];
        sw::face_flux<float>(sq, 128 * 6, t * 6, 1, P.gamma, P.igm1, (float)P.eps, out);
        sw::store_face<N, float>(flux, F, pos, out);
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

hipError_t launch_pack_mlp(const float *th, char *pk, hipStream_t st)
{
    hipLaunchKernelGGL(rt::pack_mlp_kernel, dim3(1), dim3(64), 0, st, th, pk);
    return hipGetLastError();
}

// Grid of the routed sweep of direction dir.
static void routed_grid(int dir, const FaceBox &F, long &na, long &nb)
{
    if (dir == 0) {
        if (F.cnt[0] >= sw::XSEG_MIN) {
            const long total = (long)F.cnt[0] * F.cnt[1] * F.cnt[2];
            na = (total + 255) / 256;
            nb = 1;
        } else {
            sw::sweep_tiles<0, 4>(F, na, nb);
        }
    } else {
        const long npos = (long)F.cnt[0] * F.cnt[dir == 1 ? 2 : 1];
        na = (npos + rt::YZ_PW - 1) / rt::YZ_PW;
        nb = (F.cnt[dir] + 256 / rt::YZ_PW - 1) / (256 / rt::YZ_PW);
    }
}

long routed_sweep_blocks(int dir, const FaceBox &F)
{
    long na, nb;
    routed_grid(dir, F, na, nb);
    return na * nb;
}

long routed_queue_capacity(int dir, const FaceBox &F)
{
    return (routed_sweep_blocks(dir, F) + rt::QREG - 1) / rt::QREG * 256;
}

hipError_t launch_routed_sweep(int dir, const float *u, float *flux, const Geom &G, const FaceBox &F,
                              const Phys &P, const char *pk, float thr, int force, int32_t *nsmooth,
                              unsigned long long *queue, int32_t *qcount, unsigned char *mask, int reuse,
                              const XFuse<float> *xf, hipStream_t st)
{
    const bool fused = xf != nullptr;
    if (fused && (dir != 0 || F.cnt[0] < sw::XSEG_MIN || !(G.act[0] && G.act[1] && G.act[2])))
        return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(qcount, 0, sizeof(int32_t) * rt::QREG, st);
    if (e != hipSuccess) return e;
    long na, nb;
    routed_grid(dir, F, na, nb);
    const long cap = routed_queue_capacity(dir, F);
    const dim3 grid((unsigned)na, (unsigned)nb), blk(64, 4), qgrid(32, rt::QREG), qblk(128);
    const XFuse<float> nofuse{};
    switch (dir) {
    case 0:
        if (fused)
            hipLaunchKernelGGL((rt::routed_sweep_kernel<0, true>), grid, blk, 0, st, u, flux, G, F, P, pk, thr,
                               force, nsmooth, queue, qcount, cap, mask, reuse, *xf);
        else
            hipLaunchKernelGGL((rt::routed_sweep_kernel<0, false>), grid, blk, 0, st, u, flux, G, F, P, pk, thr,
                               force, nsmooth, queue, qcount, cap, mask, reuse, nofuse);
        if (force == 0)
            hipLaunchKernelGGL(rt::troubled_kernel<0>, qgrid, qblk, 0, st, u, flux, G, F, P, queue, qcount, cap);
        if (fused && force == 0)
            hipLaunchKernelGGL(rt::xfix_queue_kernel, qgrid, qblk, 0, st, flux, G, F, *xf, queue, qcount, cap,
                               mask);
        if (fused && na > 1)
            hipLaunchKernelGGL(rt::xfix_bound_kernel, dim3((unsigned)((na - 1 + 255) / 256)), dim3(256), 0, st,
                               flux, G, F, *xf, mask, force, na);
        break;
    case 1:
        hipLaunchKernelGGL((rt::routed_sweep_kernel<1, false>), grid, blk, 0, st, u, flux, G, F, P, pk, thr, force,
                           nsmooth, queue, qcount, cap, mask, reuse, nofuse);
        if (force == 0)
            hipLaunchKernelGGL(rt::troubled_kernel<1>, qgrid, qblk, 0, st, u, flux, G, F, P, queue, qcount, cap);
        break;
    default:
        hipLaunchKernelGGL((rt::routed_sweep_kernel<2, false>), grid, blk, 0, st, u, flux, G, F, P, pk, thr, force,
                           nsmooth, queue, qcount, cap, mask, reuse, nofuse);
        if (force == 0)
            hipLaunchKernelGGL(rt::troubled_kernel<2>, qgrid, qblk, 0, st, u, flux, G, F, P, queue, qcount, cap);
        break;
    }
    return hipGetLastError();
}

}  // namespace ww
