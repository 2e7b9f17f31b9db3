// mlp.hip -- learned distance correction (an extension; the paper's distance
// comes from the GP alone).
//
// A 7-64-64-64-1 network with GELU (erf form, Hendrycks and Gimpel 2016)
// maps standardised features [d, log v, o, grad d (3), log(1 + n_local)] of a
// query to a residual r; the corrected distance is d + r where the query is
// valid and its GP variance is at most the gate, d elsewhere.  Training
// minimises the mean squared error of r against (truth - d) with Adam
// (Kingma and Ba 2015), on FP32 master weights.
//
// Kernels: the dense layers run on BF16 MFMA (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation).  One wavefront takes 32 samples: activations live in
// LDS as BF16 in the operand layouts of the next product ([sample][feature]
// for the forward B operand, [feature][sample] for the weight-gradient B
// operand), pre-activations stay in VGPRs in the accumulator layout.  The
// training kernel writes one FP32 gradient record per wavefront; a second
// kernel sums the records in wavefront order (deterministic) and applies
// Adam, a third repacks the BF16 copies of the weights.
//
// MFMA 16x16x32 BF16 lane layout (lane l, lr = l % 16, lg = l / 16):
//   A[m][k]: lane m + 16 (k / 8), element k % 8   (8 consecutive k)
//   B[k][n]: lane n + 16 (k / 8), element k % 8
//   D[m][n]: lane n + 16 (m / 4), element m % 4
#include "gpdf_internal.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace gpdf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kH = 64;       // hidden width
constexpr int kF = 7;        // features
constexpr int kS = 32;       // samples per wavefront
constexpr int kK1 = 32;      // layer-1 inputs, zero-padded to one MFMA K step
constexpr int kMaxBatch = 16384;
constexpr int kMaxWaves = kMaxBatch / kS;

// flat parameters (row-major W[out][in]), the layout of the ABI
constexpr int oW1 = 0, oB1 = oW1 + kH * kF, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH * kH, oW4 = oB3 + kH, oB4 = oW4 + kH, kNP = oB4 + 1;
static_assert(kNP == GPDF_MLP_NPARAM, "parameter count");

// BF16 copies of the weight matrices (in elements): W1 padded to [64][32],
// W2 and W3 as stored, and their transposes for the backward products
constexpr int pW1 = 0, pW2 = pW1 + kH * kK1, pW3 = pW2 + kH * kH, pW2T = pW3 + kH * kH,
              pW3T = pW2T + kH * kH, kPack = pW3T + kH * kH;

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * kInvSqrt2)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.f + erff(x * kInvSqrt2)) + x * expf(-0.5f * x * x) * kInvSqrt2Pi;
}

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// sum over the 16 lanes of a row group (lanes with equal l / 16)
__device__ __forceinline__ float sum16(float v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct MlpView {
    const float *w;        // FP32 master weights (biases and W4 are read here)
    const __bf16 *pk;      // BF16 copies
    const float *norm;     // mean[7], std[7]
};

// raw features of one query from the GP outputs
__device__ __forceinline__ void raw_features(const float *dist, const float *var, const float *grad,
                                             const float *aux, int64_t i, float *f) {
    f[0] = dist[i];
    f[1] = logf(var[i]);
    f[2] = aux[3 * i];
    f[3] = grad[3 * i];
    f[4] = grad[3 * i + 1];
    f[5] = grad[3 * i + 2];
    f[6] = log1pf(aux[3 * i + 2]);
}

// LDS of one wavefront
struct __align__(16) MlpLds {
    __bf16 X0[kS][kK1];      // standardised inputs [s][k], k >= 7 zero
    __bf16 X0T[16][kS];      // [k][s], rows >= 7 zero
    __bf16 A1[kS][kH], A2[kS][kH];      // activations [s][f]
    __bf16 A1T[kH][kS], A2T[kH][kS];    // [f][s]
    __bf16 GT[kH][kS];       // gradient of a pre-activation [o][s]
    __bf16 GS[kS][kH];       // [s][o]
};

// lanes 0..31 write the standardised features of sample s = lane (zero when
// the sample is absent)
__device__ __forceinline__ void put_inputs(MlpLds &S, int lane, bool have, const float *f,
                                           const float *norm) {
    if (lane < kS) {
#pragma unroll
        for (int k = 0; k < kK1; ++k) {
            float z = 0.f;
            if (k < kF && have) z = (f[k] - norm[k]) / norm[kF + k];
            S.X0[lane][k] = (__bf16)z;
            if (k < 16) S.X0T[k][lane] = (__bf16)z;
        }
    }
}

// GELU of the accumulator tiles into A[s][f] (and A^T when wanted)
template <bool T>
__device__ __forceinline__ void put_act(__bf16 (*A)[kH], __bf16 (*AT)[kS], const f32x4 (&p)[4][2],
                                        int lr, int lg) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = 16 * mt + 4 * lg + e, s = 16 * nt + lr;
                const __bf16 a = (__bf16)gelu(p[mt][nt][e]);
                A[s][o] = a;
                if constexpr (T) AT[o][s] = a;
            }
}

// layer 1: p1 = W1 x + b1
__device__ __forceinline__ void layer1(const MlpLds &S, const MlpView &V, int lr, int lg, f32x4 (&p)[4][2]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8 a = ld8(V.pk + pW1 + (16 * mt + lr) * kK1 + 8 * lg);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const bf16x8 b = ld8(&S.X0[16 * nt + lr][8 * lg]);
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma(a, b, c);
#pragma unroll
            for (int e = 0; e < 4; ++e) c[e] += V.w[oB1 + 16 * mt + 4 * lg + e];
            p[mt][nt] = c;
        }
    }
}

// hidden layer: p = W x + b over the 64 activations in A[s][f]
__device__ __forceinline__ void layer_h(const __bf16 (*A)[kH], const __bf16 *W, const float *b, int lr,
                                        int lg, f32x4 (&p)[4][2]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
                c = mfma(ld8(W + (16 * mt + lr) * kH + 32 * kt + 8 * lg), ld8(&A[16 * nt + lr][32 * kt + 8 * lg]), c);
#pragma unroll
            for (int e = 0; e < 4; ++e) c[e] += b[16 * mt + 4 * lg + e];
            p[mt][nt] = c;
        }
}

// forward of the 32 samples staged in S.X0; returns r for sample 16 nt + lr
// in every row group
__device__ __forceinline__ void forward(MlpLds &S, const MlpView &V, int lr, int lg, f32x4 (&p1)[4][2],
                                        f32x4 (&p2)[4][2], f32x4 (&p3)[4][2], float (&r)[2]) {
    layer1(S, V, lr, lg, p1);
    put_act<true>(S.A1, S.A1T, p1, lr, lg);
    __syncthreads();
    layer_h(S.A1, V.pk + pW2, V.w + oB2, lr, lg, p2);
    put_act<true>(S.A2, S.A2T, p2, lr, lg);
    __syncthreads();
    layer_h(S.A2, V.pk + pW3, V.w + oB3, lr, lg, p3);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        float part = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int e = 0; e < 4; ++e) part += V.w[oW4 + 16 * mt + 4 * lg + e] * gelu(p3[mt][nt][e]);
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        r[nt] = part + V.w[oB4];
    }
}

// gradient of a hidden pre-activation into GT[o][s] and GS[s][o]; the bias
// gradient (sum over samples) into rec[ob + o]
__device__ __forceinline__ void put_grad(MlpLds &S, const f32x4 (&g)[4][2], float *rec, int ob, int lr,
                                         int lg) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int o = 16 * mt + 4 * lg + e;
            float sb = 0.f;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int s = 16 * nt + lr;
                const __bf16 v = (__bf16)g[mt][nt][e];
                S.GT[o][s] = v;
                S.GS[s][o] = v;
                sb += g[mt][nt][e];
            }
            sb = sum16(sb);
            if (lr == 0) rec[ob + o] = sb;
        }
}

// weight gradient gW[o][in] = sum_s GT[o][s] AT[in][s] for 16 * nin inputs
__device__ __forceinline__ void weight_grad(const MlpLds &S, const __bf16 (*AT)[kS], int nin_tiles, int nin,
                                            float *rec, int ow, int lr, int lg) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8 a = ld8(&S.GT[16 * mt + lr][8 * lg]);
        for (int nt = 0; nt < nin_tiles; ++nt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma(a, ld8(&AT[16 * nt + lr][8 * lg]), c);
            const int in = 16 * nt + lr;
            if (in < nin) {
#pragma unroll
                for (int e = 0; e < 4; ++e) rec[ow + (16 * mt + 4 * lg + e) * nin + in] = c[e];
            }
        }
    }
}

// gradient of the previous layer's pre-activation: (W^T g) * gelu'(p)
__device__ __forceinline__ void back_prop(const MlpLds &S, const __bf16 *WT, const f32x4 (&p)[4][2], int lr,
                                          int lg, f32x4 (&g)[4][2]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
                c = mfma(ld8(WT + (16 * mt + lr) * kH + 32 * kt + 8 * lg), ld8(&S.GS[16 * nt + lr][32 * kt + 8 * lg]),
                         c);
#pragma unroll
            for (int e = 0; e < 4; ++e) c[e] *= gelu_d(p[mt][nt][e]);
            g[mt][nt] = c;
        }
}

// Forward and backward of one 32-sample slice of a mini-batch.  Batch
// position i maps to sample (a i + b) mod n (a coprime to n: a permutation).
// Writes the gradient of (1/ntot) sum (r - target)^2 into rec[wave] and the
// slice's sum of squared errors into loss[wave].
__global__ __launch_bounds__(64) void k_mlp_step(const float *__restrict__ feat, const float *__restrict__ tgt,
                                                 int64_t n, uint64_t pa, uint64_t pb, int64_t start, int64_t cnt,
                                                 float inv_ntot, MlpView V, float *__restrict__ rec_all,
                                                 float *__restrict__ loss) {
    __shared__ MlpLds S;
    const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
    const int64_t s0 = int64_t(blockIdx.x) * kS;
    float *rec = rec_all + int64_t(blockIdx.x) * kNP;
    // stage inputs
    {
        float f[kF] = {};
        const bool have = lane < kS && s0 + lane < cnt;
        float t = 0.f;
        if (have) {
            const uint64_t g = (pa * uint64_t(start + s0 + lane) + pb) % uint64_t(n);
#pragma unroll
            for (int k = 0; k < kF; ++k) f[k] = feat[int64_t(g) * kF + k];
            t = tgt[g];
        }
        put_inputs(S, lane, have, f, V.norm);
        __syncthreads();
        // targets of samples lr and 16 + lr, in every row group (FP32)
        const float tt0 = __shfl(t, lr, 64), tt1 = __shfl(t, 16 + lr, 64);
        f32x4 p1[4][2], p2[4][2], p3[4][2];
        float r[2];
        forward(S, V, lr, lg, p1, p2, p3, r);
        // loss and dL/dr
        float gr[2], lsum = 0.f;
        const float tt[2] = {tt0, tt1};
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const bool valid = s0 + 16 * nt + lr < cnt;
            const float e = r[nt] - tt[nt];
            gr[nt] = valid ? 2.f * e * inv_ntot : 0.f;
            if (valid && lg == 0) lsum += e * e;
        }
        lsum = wave_sum(lsum);
        if (lane == 0) loss[blockIdx.x] = lsum;
        // output layer: gW4[o] = sum_s gr[s] a3[o][s], gb4 = sum_s gr[s]
        f32x4 g3[4][2];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = 16 * mt + 4 * lg + e;
                const float w4 = V.w[oW4 + o];
                float q = 0.f;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const float x = p3[mt][nt][e];
                    q += gr[nt] * gelu(x);
                    g3[mt][nt][e] = gr[nt] * w4 * gelu_d(x);
                }
                q = sum16(q);
                if (lr == 0) rec[oW4 + o] = q;
            }
        {
            float q = lg == 0 ? gr[0] + gr[1] : 0.f;
            q = wave_sum(q);
            if (lane == 0) rec[oB4] = q;
        }
        // layer 3
        __syncthreads();
        put_grad(S, g3, rec, oB3, lr, lg);
        __syncthreads();
        weight_grad(S, S.A2T, 4, kH, rec, oW3, lr, lg);
        f32x4 g2[4][2];
        back_prop(S, V.pk + pW3T, p2, lr, lg, g2);
        // layer 2
        __syncthreads();
        put_grad(S, g2, rec, oB2, lr, lg);
        __syncthreads();
        weight_grad(S, S.A1T, 4, kH, rec, oW2, lr, lg);
        f32x4 g1[4][2];
        back_prop(S, V.pk + pW2T, p1, lr, lg, g1);
        // layer 1
        __syncthreads();
        put_grad(S, g1, rec, oB1, lr, lg);
        __syncthreads();
        weight_grad(S, S.X0T, 1, kF, rec, oW1, lr, lg);
    }
}

// sum of the per-wavefront records in wavefront order; optional Adam step
// (bias-corrected, beta = 0.9 / 0.999, eps = 1e-8) on the master weights
__global__ void k_mlp_reduce(const float *__restrict__ rec, int nrec, float *__restrict__ gacc, int accumulate,
                             float *__restrict__ w, float *__restrict__ m, float *__restrict__ v, int adam,
                             float lr, float c1, float c2, const float *__restrict__ loss_rec,
                             float *__restrict__ loss_acc) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        float l = 0.f;
        for (int i = 0; i < nrec; ++i) l += loss_rec[i];
        *loss_acc += l;
    }
    if (p >= kNP) return;
    float g = 0.f;
    for (int i = 0; i < nrec; ++i) g += rec[int64_t(i) * kNP + p];
    if (accumulate) g += gacc[p];
    gacc[p] = g;
    if (adam) {
        const float mm = 0.9f * m[p] + 0.1f * g;
        const float vv = 0.999f * v[p] + 0.001f * g * g;
        m[p] = mm;
        v[p] = vv;
        w[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
    }
}

// BF16 copies of the weight matrices from the master weights
__global__ void k_mlp_pack(const float *__restrict__ w, __bf16 *__restrict__ pk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kH * kK1) {
        const int o = i / kK1, k = i % kK1;
        pk[pW1 + i] = (__bf16)(k < kF ? w[oW1 + o * kF + k] : 0.f);
    }
    if (i < kH * kH) {
        const int o = i / kH, k = i % kH;
        pk[pW2 + i] = (__bf16)w[oW2 + i];
        pk[pW3 + i] = (__bf16)w[oW3 + i];
        pk[pW2T + k * kH + o] = (__bf16)w[oW2 + i];
        pk[pW3T + k * kH + o] = (__bf16)w[oW3 + i];
    }
}

__global__ void k_mlp_features(const float *__restrict__ dist, const float *__restrict__ var,
                               const float *__restrict__ grad, const float *__restrict__ aux, int64_t n,
                               float *__restrict__ feat) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[kF];
    raw_features(dist, var, grad, aux, i, f);
#pragma unroll
    for (int k = 0; k < kF; ++k) feat[i * kF + k] = f[k];
}

// per-block partial sums of each feature and its square (FP64) for the
// standardisation of a training set
__global__ void k_mlp_moments(const float *__restrict__ feat, int64_t n, double *__restrict__ part) {
    __shared__ double sh[2 * kF][4];
    double s[kF] = {}, q[kF] = {};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
#pragma unroll
        for (int k = 0; k < kF; ++k) {
            const double x = feat[i * kF + k];
            s[k] += x;
            q[k] += x * x;
        }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kF; ++k) {
        double a = s[k], b = q[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o, 64);
            b += __shfl_xor(b, o, 64);
        }
        if (lane == 0) { sh[k][w] = a; sh[kF + k][w] = b; }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kF)
        part[int64_t(blockIdx.x) * 2 * kF + threadIdx.x] =
            sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
}

// Inference: residual r for raw features (feat != NULL) or for the outputs
// of a query, and the gate: out = d + r where valid and var <= gate.
__global__ __launch_bounds__(64) void k_mlp_infer(const float *__restrict__ feat, const float *__restrict__ dist,
                                                  const float *__restrict__ var, const float *__restrict__ grad,
                                                  const float *__restrict__ aux, const uint8_t *__restrict__ valid,
                                                  int64_t n, float gate, MlpView V, float *__restrict__ r_out,
                                                  float *__restrict__ d_out, unsigned long long *__restrict__ spread) {
    __shared__ MlpLds S;
    const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
    const int64_t s0 = int64_t(blockIdx.x) * kS;
    const int64_t i = s0 + lane;
    const bool have = lane < kS && i < n;
    float f[kF] = {};
    bool use = have;
    if (have) {
        if (feat) {
#pragma unroll
            for (int k = 0; k < kF; ++k) f[k] = feat[i * kF + k];
        } else {
            use = valid[i] && var[i] <= gate;
            if (use) raw_features(dist, var, grad, aux, i, f);
        }
    }
    put_inputs(S, lane, use, f, V.norm);
    __syncthreads();
    f32x4 p1[4][2], p2[4][2], p3[4][2];
    float r[2];
    forward(S, V, lr, lg, p1, p2, p3, r);
    // lane l < 32 holds r of samples l % 16 and 16 + l % 16: sample l is r[l / 16]
    const float rl = (lane & 16) ? r[1] : r[0];
    if (have) {
        if (r_out) r_out[i] = rl;
        if (d_out && use) d_out[i] = dist[i] + rl;
    }
    if (d_out) {
        const uint64_t mb = __ballot(have && use);
        if (lane == 0 && mb) spread_add(spread, ST_GATED, (unsigned long long)__popcll(mb));
    }
}

inline unsigned blocks(int64_t n, int t) { return unsigned(std::max<int64_t>(1, (n + t - 1) / t)); }

// counter-based generator for the initial weights: SplitMix64 (Steele,
// Lea and Flood 2014)
uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

gpdf_status mlp_alloc(gpdf_ctx *c) {
    if (c->d_mlp_w) return GPDF_OK;
    hipError_t e;
    if ((e = hipMalloc((void **)&c->d_mlp_w, sizeof(float) * kNP)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_m, sizeof(float) * kNP)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_v, sizeof(float) * kNP)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_g, sizeof(float) * kNP)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_rec, sizeof(float) * kNP * int64_t(kMaxWaves))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_pack, sizeof(__bf16) * kPack)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_norm, sizeof(float) * 2 * kF)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_loss, sizeof(float) * (kMaxWaves + 1))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_mlp_mom, sizeof(double) * 2 * kF * 1024)) != hipSuccess)
        return hip_fail(c, e, "mlp: allocate");
    return GPDF_OK;
}

MlpView view(gpdf_ctx *c) {
    return MlpView{c->d_mlp_w, reinterpret_cast<const __bf16 *>(c->d_mlp_pack), c->d_mlp_norm};
}

gpdf_status pack(gpdf_ctx *c) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(blocks(kH * kH, 256)), dim3(256), 0, c->stream, c->d_mlp_w,
                       reinterpret_cast<__bf16 *>(c->d_mlp_pack));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "mlp: pack");
}

gpdf_status zero_adam(gpdf_ctx *c) {
    fill_u32(reinterpret_cast<uint32_t *>(c->d_mlp_m), 0u, kNP, c->stream);
    fill_u32(reinterpret_cast<uint32_t *>(c->d_mlp_v), 0u, kNP, c->stream);
    c->mlp_step = 0;
    return GPDF_OK;
}

// one pass of k_mlp_step + k_mlp_reduce over batch positions [start, start + cnt)
gpdf_status mlp_batch(gpdf_ctx *c, const float *feat, const float *tgt, int64_t n, uint64_t pa, uint64_t pb,
                      int64_t start, int64_t cnt, float inv_ntot, bool accumulate, bool adam, float lr) {
    const int nw = int((cnt + kS - 1) / kS);
    hipLaunchKernelGGL(k_mlp_step, dim3(nw), dim3(64), 0, c->stream, feat, tgt, n, pa, pb, start, cnt, inv_ntot,
                       view(c), c->d_mlp_rec, c->d_mlp_loss);
    float c1 = 1.f, c2 = 1.f;
    if (adam) {
        ++c->mlp_step;
        c1 = float(1.0 / (1.0 - std::pow(0.9, double(c->mlp_step))));
        c2 = float(1.0 / (1.0 - std::pow(0.999, double(c->mlp_step))));
    }
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks(kNP, 256)), dim3(256), 0, c->stream, c->d_mlp_rec, nw,
                       c->d_mlp_g, accumulate ? 1 : 0, c->d_mlp_w, c->d_mlp_m, c->d_mlp_v, adam ? 1 : 0, lr, c1,
                       c2, c->d_mlp_loss, c->d_mlp_loss + kMaxWaves);
    if (adam) return pack(c);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "mlp: batch");
}

gpdf_status need_ready(gpdf_ctx *c) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (!c->mlp_ready) return fail(c, GPDF_E_INVALID_ARG, "learned correction: no weights (gpdf_mlp_init)");
    return GPDF_OK;
}

uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) { const uint64_t t = a % b; a = b; b = t; }
    return a;
}

}  // namespace

gpdf_status mlp_apply(gpdf_ctx *c, const float *dist, const float *var, const float *grad, const float *aux,
                      const uint8_t *valid, int64_t m, float *out) {
    gpdf_status st = need_ready(c);
    if (st != GPDF_OK) return st;
    if (!var || !grad || !aux)
        return fail(c, GPDF_E_INVALID_ARG, "learned correction needs the variance, gradient and aux outputs");
    stage_begin(c, GPDF_MS_MLP);
    fill_u64(c->d_stat + ST_GATED, 0ull, 1, c->stream);
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks(m, kS)), dim3(64), 0, c->stream, nullptr, dist, var, grad, aux,
                       valid, m, float(c->p.mlp_gate), view(c), nullptr, out, c->d_spread);
    fold_stats(c->d_spread, c->d_stat, c->stream);
    stage_end(c, GPDF_MS_MLP);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "mlp: apply");
}

}  // namespace gpdf

using namespace gpdf;

extern "C" gpdf_status gpdf_mlp_init(gpdf_ctx *c, uint64_t seed) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    gpdf_status st = mlp_alloc(c);
    if (st != GPDF_OK) return st;
    // W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases 0, identity standardisation
    std::vector<float> w(kNP, 0.f);
    uint64_t x = seed;
    auto fill = [&](int off, int nout, int nin) {
        const double b = 1.0 / std::sqrt(double(nin));
        for (int i = 0; i < nout * nin; ++i)
            w[off + i] = float((double(splitmix64(x) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * b);
    };
    fill(oW1, kH, kF);
    fill(oW2, kH, kH);
    fill(oW3, kH, kH);
    fill(oW4, 1, kH);
    float norm[2 * kF];
    for (int k = 0; k < kF; ++k) { norm[k] = 0.f; norm[kF + k] = 1.f; }
    hipError_t e;
    if ((e = hipMemcpyAsync(c->d_mlp_w, w.data(), sizeof(float) * kNP, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(c->d_mlp_norm, norm, sizeof(norm), hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "mlp_init");
    zero_adam(c);
    c->mlp_ready = true;
    return pack(c);
}

extern "C" gpdf_status gpdf_mlp_set_weights(gpdf_ctx *c, const float *h_w, int64_t n) {
    if (!c || !h_w) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (n != kNP) return fail(c, GPDF_E_INVALID_ARG, "mlp_set_weights: expected 8897 parameters");
    gpdf_status st = mlp_alloc(c);
    if (st != GPDF_OK) return st;
    hipError_t e;
    if ((e = hipMemcpyAsync(c->d_mlp_w, h_w, sizeof(float) * kNP, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "mlp_set_weights");
    if (!c->mlp_ready) {
        float norm[2 * kF];
        for (int k = 0; k < kF; ++k) { norm[k] = 0.f; norm[kF + k] = 1.f; }
        if ((e = hipMemcpy(c->d_mlp_norm, norm, sizeof(norm), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(c, e, "mlp_set_weights");
    }
    zero_adam(c);
    c->mlp_ready = true;
    return pack(c);
}

extern "C" gpdf_status gpdf_mlp_get_weights(gpdf_ctx *c, float *h_w, int64_t cap) {
    gpdf_status st = need_ready(c);
    if (st != GPDF_OK) return st;
    if (!h_w || cap < kNP) return fail(c, GPDF_E_INVALID_ARG, "mlp_get_weights: buffer too small");
    hipError_t e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess ||
        (e = hipMemcpy(h_w, c->d_mlp_w, sizeof(float) * kNP, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "mlp_get_weights");
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_mlp_set_norm(gpdf_ctx *c, const float *h_mean, const float *h_std) {
    gpdf_status st = need_ready(c);
    if (st != GPDF_OK) return st;
    if (!h_mean || !h_std) return fail(c, GPDF_E_INVALID_ARG, "mlp_set_norm: null");
    float norm[2 * kF];
    for (int k = 0; k < kF; ++k) {
        if (!std::isfinite(h_mean[k]) || !(h_std[k] > 0.f) || !std::isfinite(h_std[k]))
            return fail(c, GPDF_E_INVALID_ARG, "mlp_set_norm: mean must be finite and std positive");
        norm[k] = h_mean[k];
        norm[kF + k] = h_std[k];
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(c->d_mlp_norm, norm, sizeof(norm), hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "mlp_set_norm");
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_mlp_get_norm(gpdf_ctx *c, float *h_mean, float *h_std) {
    gpdf_status st = need_ready(c);
    if (st != GPDF_OK) return st;
    if (!h_mean || !h_std) return fail(c, GPDF_E_INVALID_ARG, "mlp_get_norm: null");
    float norm[2 * kF];
    hipError_t e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess ||
        (e = hipMemcpy(norm, c->d_mlp_norm, sizeof(norm), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "mlp_get_norm");
    for (int k = 0; k < kF; ++k) { h_mean[k] = norm[k]; h_std[k] = norm[kF + k]; }
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_mlp_features(gpdf_ctx *c, const float *d_dist, const float *d_var,
                                         const float *d_grad, const float *d_aux, int64_t n, float *d_feat) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (n < 0) return fail(c, GPDF_E_INVALID_ARG, "mlp_features: n < 0");
    if (n == 0) return GPDF_OK;
    if (!d_dist || !d_var || !d_grad || !d_aux || !d_feat) return fail(c, GPDF_E_INVALID_ARG, "mlp_features: null");
    hipLaunchKernelGGL(k_mlp_features, dim3(blocks(n, 256)), dim3(256), 0, c->stream, d_dist, d_var, d_grad, d_aux,
                       n, d_feat);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "mlp_features");
}

extern "C" gpdf_status gpdf_mlp_forward(gpdf_ctx *c, const float *d_feat, int64_t n, float *d_r) {
    gpdf_status st = need_ready(c);
    if (st != GPDF_OK) return st;
    if (n < 0) return fail(c, GPDF_E_INVALID_ARG, "mlp_forward: n < 0");
    if (n == 0) return GPDF_OK;
    if (!d_feat || !d_r) return fail(c, GPDF_E_INVALID_ARG, "mlp_forward: null");
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks(n, kS)), dim3(64), 0, c->stream, d_feat, nullptr, nullptr, nullptr,
                       nullptr, nullptr, n, 0.f, view(c), d_r, nullptr, c->d_spread);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "mlp_forward");
}

extern "C" gpdf_status gpdf_mlp_grad(gpdf_ctx *c, const float *d_feat, const float *d_target, int64_t n,
                                     float *d_grad, float *h_loss) {
    gpdf_status st = need_ready(c);
    if (st != GPDF_OK) return st;
    if (n < 1 || !d_feat || !d_target) return fail(c, GPDF_E_INVALID_ARG, "mlp_grad: empty or null input");
    if (n > (int64_t(1) << 31)) return fail(c, GPDF_E_CAPACITY, "mlp_grad: n too large");
    fill_u32(reinterpret_cast<uint32_t *>(c->d_mlp_loss + kMaxWaves), 0u, 1, c->stream);
    const float inv = float(1.0 / double(n));
    for (int64_t s = 0; s < n; s += kMaxBatch) {
        st = mlp_batch(c, d_feat, d_target, n, 1, 0, s, std::min<int64_t>(kMaxBatch, n - s), inv, s > 0, false,
                       0.f);
        if (st != GPDF_OK) return st;
    }
    hipError_t e;
    float loss = 0.f;
    if (d_grad &&
        (e = hipMemcpyAsync(d_grad, c->d_mlp_g, sizeof(float) * kNP, hipMemcpyDeviceToDevice, c->stream)) !=
            hipSuccess)
        return hip_fail(c, e, "mlp_grad: copy");
    if ((e = hipMemcpyAsync(&loss, c->d_mlp_loss + kMaxWaves, 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "mlp_grad: loss");
    if (h_loss) *h_loss = float(double(loss) / double(n));
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_mlp_train(gpdf_ctx *c, const float *d_feat, const float *d_target, int64_t n,
                                      int32_t epochs, int32_t batch, float lr, uint64_t seed, float *h_loss) {
    gpdf_status st = need_ready(c);
    if (st != GPDF_OK) return st;
    if (n < 1 || !d_feat || !d_target) return fail(c, GPDF_E_INVALID_ARG, "mlp_train: empty or null input");
    if (n > (int64_t(1) << 31)) return fail(c, GPDF_E_CAPACITY, "mlp_train: n too large");
    if (epochs < 1 || batch < 1 || batch > kMaxBatch || !(lr > 0.f) || !std::isfinite(lr))
        return fail(c, GPDF_E_INVALID_ARG, "mlp_train: epochs >= 1, 1 <= batch <= 16384, lr > 0");
    hipStream_t s = c->stream;
    hipError_t e;
    // standardisation from this training set (FP64 moments)
    {
        const int nb = int(std::min<int64_t>(1024, (n + 255) / 256));
        hipLaunchKernelGGL(k_mlp_moments, dim3(nb), dim3(256), 0, s, d_feat, n, c->d_mlp_mom);
        std::vector<double> part(size_t(nb) * 2 * kF);
        if ((e = hipMemcpyAsync(part.data(), c->d_mlp_mom, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(c, e, "mlp_train: moments");
        float norm[2 * kF];
        for (int k = 0; k < kF; ++k) {
            double sm = 0.0, sq = 0.0;
            for (int b = 0; b < nb; ++b) { sm += part[size_t(b) * 2 * kF + k]; sq += part[size_t(b) * 2 * kF + kF + k]; }
            const double mean = sm / double(n);
            const double var = std::max(sq / double(n) - mean * mean, 0.0);
            if (!std::isfinite(mean) || !std::isfinite(var))
                return fail(c, GPDF_E_INVALID_ARG, "mlp_train: non-finite features");
            norm[k] = float(mean);
            norm[kF + k] = float(std::max(std::sqrt(var), 1e-6));
        }
        if ((e = hipMemcpyAsync(c->d_mlp_norm, norm, sizeof(norm), hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(c, e, "mlp_train: norm");
    }
    // epochs: order (a i + b) mod n with a coprime to n, drawn from the seed
    uint64_t x = seed;
    float last = 0.f;
    for (int ep = 0; ep < epochs; ++ep) {
        uint64_t a = 1, b = 0;
        if (n > 1) {
            a = splitmix64(x) % uint64_t(n);
            if (a == 0) a = 1;
            while (gcd64(a, uint64_t(n)) != 1) a = a + 1 < uint64_t(n) ? a + 1 : 1;
            b = splitmix64(x) % uint64_t(n);
        }
        fill_u32(reinterpret_cast<uint32_t *>(c->d_mlp_loss + kMaxWaves), 0u, 1, s);
        for (int64_t st0 = 0; st0 < n; st0 += batch) {
            const int64_t cnt = std::min<int64_t>(batch, n - st0);
            st = mlp_batch(c, d_feat, d_target, n, a, b, st0, cnt, float(1.0 / double(cnt)), false, true, lr);
            if (st != GPDF_OK) return st;
        }
        float l = 0.f;
        if ((e = hipMemcpyAsync(&l, c->d_mlp_loss + kMaxWaves, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(c, e, "mlp_train: loss");
        last = float(double(l) / double(n));
    }
    if (h_loss) *h_loss = last;
    return GPDF_OK;
}
