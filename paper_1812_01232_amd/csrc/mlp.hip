// Queue-ordering network: 20 -> 128 -> 128 -> 128 -> 1, GELU, bf16 weights and
// activations, FP32 accumulation on the matrix cores (MFMA 16x16x16 bf16).
//
// It predicts, for a queued cube, how much the lower bound of its children
// will exceed its own (normalised by S22).  The branch-and-bound uses the
// prediction only to order its queue; pruning and the stop test use the exact
// bounds.  Training runs here too: forward, backward through the activations,
// weight-gradient GEMMs and Adam, all on the GPU.
//
// MFMA operand layout (v_mfma_f32_16x16x16bf16_1k): lane l holds
//   A[m = l % 16][k = 4 (l / 16) + j], B[k = 4 (l / 16) + j][n = l % 16], j = 0..3,
// and receives D[m = 4 (l / 16) + j][n = l % 16].  Every tile product here is
// D = A Bt^T with A and Bt both stored row-major with K contiguous, so each
// lane loads 4 consecutive bf16 of one row of each operand.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "gosma_impl.h"

namespace gosma {

namespace {

constexpr int IN = GOSMA_MLP_FEATURES, INP = 32, HID = 128, OUTP = 16;
constexpr int oW1 = 0, ob1 = oW1 + HID * IN, oW2 = ob1 + HID, ob2 = oW2 + HID * HID, oW3 = ob2 + HID,
              ob3 = oW3 + HID * HID, oW4 = ob3 + HID, ob4 = oW4 + HID, NP = ob4 + 1;
static_assert(NP == GOSMA_MLP_PARAMS, "parameter count");
// LDS row strides (bf16 elements), padded by 8 so that the 16 rows a wave
// reads in one operand load fall in different banks
constexpr int S_H = HID + 8;
constexpr int kThreads = 256;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __host__ inline uint16_t f2bf(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __host__ inline float bf2f(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}
__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_prime(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

__device__ inline bf16x4 ld4(const uint16_t *p)
{
    bf16x4 v;
    const uint2 u = *(const uint2 *)p;       // 4 bf16, 8-byte aligned
    v[0] = (short)(u.x & 0xffff);
    v[1] = (short)(u.x >> 16);
    v[2] = (short)(u.y & 0xffff);
    v[3] = (short)(u.y >> 16);
    return v;
}
__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Device weights: bf16 copies in the layouts the kernels read, FP32 biases.
struct Weights {
    const uint16_t *W1, *W2, *W3, *W4;   // [HID][INP], [HID][HID], [HID][HID], [OUTP][HID] (row 0 real)
    const uint16_t *W2t, *W3t, *W4t;     // transposed: [HID][HID], [HID][HID], [HID][OUTP] (col 0 real)
    const float *b;                      // packed FP32 parameter vector (biases read from it)
};

struct Save {          // per-minibatch activations for the backward pass (B = stride)
    float *z1, *z2, *z3;                 // [B][HID]
    uint16_t *h0fm, *h1fm, *h2fm, *h3fm; // feature-major: [INP][B], [HID][B] x 3
    int B;
};

// One dense layer on a 16-row activation tile held in LDS:
// out[16][N] = act(in[16][K] W^T + bias), W given as rows [N][K] (global).
// The calling wave computes the output columns of tiles [nt0, nt0 + NT).
template <int K, int NT, bool GELU_>
__device__ inline void layer16(int nt0, const uint16_t *in, int ldi, const uint16_t *W, int ldw, const float *bias,
                               uint16_t *out, int ldo, float *zsave, uint16_t *hfm, int B, int rec0, int nrec)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int nt = nt0; nt < nt0 + NT; ++nt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks)
            acc = mfma(ld4(in + r * ldi + 16 * ks + 4 * g), ld4(W + (16 * nt + r) * ldw + 16 * ks + 4 * g), acc);
        const int col = 16 * nt + r;
        const float bc = bias[col];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 4 * g + j;
            const float z = acc[j] + bc;
            const float h = GELU_ ? gelu(z) : z;
            const uint16_t hb = f2bf(h);
            out[row * ldo + col] = hb;
            if (zsave) {   // padding rows of the tile store zeros for the gradient GEMMs
                if (row < nrec) zsave[(size_t)(rec0 + row) * HID + col] = z;
                hfm[(size_t)col * B + rec0 + row] = row < nrec ? hb : (uint16_t)0;
            }
        }
    }
}

// Forward pass.  X: n x IN FP32 features (record-major).  y: n outputs.  With
// a Save, also stores the pre-activations and feature-major activations
// (training).  n may be read from device memory (n_dev).  A block of four
// waves takes one 16-record tile at a time, each wave a quarter of every
// layer's output columns (the dependent chain of one tile is a quarter as
// long as with one wave per tile, and a launch has four times the waves).
__global__ __launch_bounds__(kThreads) void k_forward(Weights w, const float *__restrict__ X, int64_t n_host,
                                                      const uint32_t *n_dev, float *__restrict__ y, Save sv)
{
    extern __shared__ uint16_t lds[];
    // weights are read straight from global memory (72 KB, cache-resident);
    // LDS holds the tile's activations, 2 x [16][S_H]
    uint16_t *a0 = lds, *a1 = lds + 16 * S_H;
    const uint16_t *W1 = w.W1, *W2 = w.W2, *W3 = w.W3, *W4 = w.W4;
    const int64_t n = n_dev ? (int64_t)n_dev[0] : n_host;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int NT = HID / 16 / (kThreads / 64);   // column tiles per wave
    const int64_t ntiles = (n + 15) / 16;
    const bool train = sv.z1 != nullptr;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t rec0 = t * 16;
        const int nrec = (int)std::min<int64_t>(16, n - rec0);
        // input tile -> bf16 [16][INP] (features beyond IN and rows beyond n are zero)
        for (int i = threadIdx.x; i < 16 * INP; i += kThreads) {
            const int row = i / INP, col = i % INP;
            float v = 0.0f;
            if (row < nrec && col < IN) v = X[(rec0 + row) * IN + col];
            const uint16_t hb = f2bf(v);
            a0[row * S_H + col] = hb;
            if (train) sv.h0fm[(size_t)col * sv.B + rec0 + row] = hb;
        }
        __syncthreads();
        layer16<INP, NT, true>(NT * wave, a0, S_H, W1, INP, w.b + ob1, a1, S_H, train ? sv.z1 : nullptr, sv.h1fm,
                               sv.B, (int)rec0, nrec);
        __syncthreads();
        layer16<HID, NT, true>(NT * wave, a1, S_H, W2, HID, w.b + ob2, a0, S_H, train ? sv.z2 : nullptr, sv.h2fm,
                               sv.B, (int)rec0, nrec);
        __syncthreads();
        layer16<HID, NT, true>(NT * wave, a0, S_H, W3, HID, w.b + ob3, a1, S_H, train ? sv.z3 : nullptr, sv.h3fm,
                               sv.B, (int)rec0, nrec);
        __syncthreads();
        if (wave == 0) {
            const int r = lane & 15, g = lane >> 4;
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < HID / 16; ++ks)
                acc = mfma(ld4(a1 + r * S_H + 16 * ks + 4 * g), ld4(W4 + r * HID + 16 * ks + 4 * g), acc);
            if (r == 0) {
                const float b4 = w.b[ob4];
                for (int j = 0; j < 4; ++j)
                    if (4 * g + j < nrec) y[rec0 + 4 * g + j] = acc[j] + b4;
            }
        }
        __syncthreads();
    }
}

// Loss gradient: dy = 2 (y - target) / n for the mean squared error, stored
// in bf16 as the 16-wide (column 0) operand of the output layer; the loss sum
// accumulates in *loss.
__global__ void k_loss(const float *y, const float *target, int n, int B, uint16_t *dy_rm, uint16_t *dz4fm,
                       float *loss)
{
    float l = 0.0f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x) {
        float d = 0.0f;
        if (i < n) {
            const float e = y[i] - target[i];
            l += e * e;
            d = 2.0f * e / (float)n;
        }
        const uint16_t db = f2bf(d);
        dy_rm[(size_t)i * OUTP] = db;
        dz4fm[i] = db;
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if ((threadIdx.x & 63) == 0 && l != 0.0f) atomicAdd(loss, l);
}

// Backward through the activations: dz3, dz2, dz1 (feature-major, bf16).
__global__ __launch_bounds__(kThreads) void k_backward(Weights w, const uint16_t *__restrict__ dy_rm, Save sv,
                                                       uint16_t *dz3fm, uint16_t *dz2fm, uint16_t *dz1fm, int n)
{
    extern __shared__ uint16_t lds[];
    uint16_t *act = lds;
    const uint16_t *W4t = w.W4t, *W3t = w.W3t, *W2t = w.W2t;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    uint16_t *a0 = act + wave * 2 * 16 * S_H, *a1 = a0 + 16 * S_H;
    const int ntiles = (n + 15) / 16;
    for (int t0 = blockIdx.x * 4; t0 < ntiles; t0 += gridDim.x * 4) {
        const int t = t0 + wave;
        const bool valid = t < ntiles;
        const int rec0 = t * 16;
        const int nrec = valid ? std::min(16, n - rec0) : 0;
        // dz3 = (dy W4) * gelu'(z3): A = dy [16][16], Bt = W4t [HID][16]
        if (valid) {
            const bf16x4 a = nrec > r ? ld4(dy_rm + (size_t)(rec0 + r) * OUTP + 4 * g) : bf16x4{0, 0, 0, 0};
            for (int nt = 0; nt < HID / 16; ++nt) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                acc = mfma(a, ld4(W4t + (16 * nt + r) * OUTP + 4 * g), acc);
                const int col = 16 * nt + r;
                for (int j = 0; j < 4; ++j) {
                    const int row = 4 * g + j;
                    const float d = row < nrec ? acc[j] * gelu_prime(sv.z3[(size_t)(rec0 + row) * HID + col]) : 0.0f;
                    const uint16_t db = f2bf(d);
                    a0[row * S_H + col] = db;
                    dz3fm[(size_t)col * sv.B + rec0 + row] = db;
                }
            }
        }
        __syncthreads();
        // dz2 = (dz3 W3) * gelu'(z2), dz1 = (dz2 W2) * gelu'(z1)
        for (int layer = 0; layer < 2; ++layer) {
            const uint16_t *in = layer == 0 ? a0 : a1;
            uint16_t *out = layer == 0 ? a1 : a0;
            const uint16_t *Wt = layer == 0 ? W3t : W2t;
            const float *z = layer == 0 ? sv.z2 : sv.z1;
            uint16_t *fm = layer == 0 ? dz2fm : dz1fm;
            if (valid) {
                for (int nt = 0; nt < HID / 16; ++nt) {
                    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int ks = 0; ks < HID / 16; ++ks)
                        acc = mfma(ld4(in + r * S_H + 16 * ks + 4 * g), ld4(Wt + (16 * nt + r) * HID + 16 * ks + 4 * g),
                                   acc);
                    const int col = 16 * nt + r;
                    for (int j = 0; j < 4; ++j) {
                        const int row = 4 * g + j;
                        const float d = row < nrec ? acc[j] * gelu_prime(z[(size_t)(rec0 + row) * HID + col]) : 0.0f;
                        const uint16_t db = f2bf(d);
                        out[row * S_H + col] = db;
                        fm[(size_t)col * sv.B + rec0 + row] = db;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Weight gradients dW[out][in] = sum_r dz[out][r] h[in][r]: one wavefront per
// 16 x 16 tile, K = the minibatch.  Also the bias gradient of each out row
// (computed by the waves of the first in-tile).  Writes the packed gradient.
struct WgradJob {
    const uint16_t *dz;   // [outs][B]
    const uint16_t *h;    // [ins][B]
    int outs_real, ins_real, ins_tiles, w_off, b_off;
};

__global__ __launch_bounds__(kThreads) void k_wgrad(WgradJob j1, WgradJob j2, WgradJob j3, WgradJob j4, int B,
                                                    int n, float *grad)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    int tile = blockIdx.x * 4 + wave;
    const WgradJob *jobs[4] = {&j1, &j2, &j3, &j4};
    for (int q = 0; q < 4; ++q) {
        const WgradJob &J = *jobs[q];
        const int nt = ((J.outs_real + 15) / 16) * J.ins_tiles;
        if (tile >= nt) {
            tile -= nt;
            continue;
        }
        const int mt = tile / J.ins_tiles, it = tile % J.ins_tiles;
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        float bsum = 0.0f;
        const uint16_t *A = J.dz + (size_t)(16 * mt + r) * B;
        const uint16_t *Bt = J.h + (size_t)(16 * it + r) * B;
        for (int k0 = 0; k0 < n; k0 += 16) {
            const bf16x4 a = ld4(A + k0 + 4 * g);
            acc = mfma(a, ld4(Bt + k0 + 4 * g), acc);
            if (it == 0)
                for (int e = 0; e < 4; ++e) bsum += bf2f((uint16_t)a[e]);
        }
        for (int e = 0; e < 4; ++e) {
            const int o = 16 * mt + 4 * g + e, i = 16 * it + r;
            if (o < J.outs_real && i < J.ins_real) grad[J.w_off + o * J.ins_real + i] = acc[e];
        }
        if (it == 0) {
            // lanes r, r + 16, r + 32, r + 48 hold the partial sums of out row 16 mt + r
            bsum += __shfl_xor(bsum, 16, 64);
            bsum += __shfl_xor(bsum, 32, 64);
            if (g == 0 && 16 * mt + r < J.outs_real) grad[J.b_off + 16 * mt + r] = bsum;
        }
        return;
    }
}

__global__ void k_adam(float *p, const float *grad, float *m, float *v, int np, float lr, float b1, float b2,
                       float c1, float c2, float eps)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// FP32 parameters -> the bf16 layouts of Weights.
__global__ void k_pack(const float *p, uint16_t *W1, uint16_t *W2, uint16_t *W3, uint16_t *W4, uint16_t *W2t,
                       uint16_t *W3t, uint16_t *W4t)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < HID * HID; i += gridDim.x * blockDim.x) {
        const int o = i / HID, c = i % HID;
        const uint16_t w2 = f2bf(p[oW2 + i]), w3 = f2bf(p[oW3 + i]);
        W2[i] = w2;
        W3[i] = w3;
        W2t[c * HID + o] = w2;
        W3t[c * HID + o] = w3;
        if (i < HID * INP) {
            const int oo = i / INP, cc = i % INP;
            W1[i] = cc < IN ? f2bf(p[oW1 + oo * IN + cc]) : 0;
        }
        if (i < OUTP * HID) {
            const int oo = i / HID, cc = i % HID;
            const uint16_t w4 = oo == 0 ? f2bf(p[oW4 + cc]) : 0;
            W4[i] = w4;
            W4t[cc * OUTP + oo] = w4;
        }
    }
}

// Gather a minibatch of records (21 floats: features, target) by index.
__global__ void k_gather(const float *records, const uint32_t *perm, int64_t off, int n, float *X, float *t)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * (IN + 1); i += gridDim.x * blockDim.x) {
        const int r = i / (IN + 1), c = i % (IN + 1);
        const float v = records[(size_t)perm[off + r] * (IN + 1) + c];
        if (c < IN)
            X[(size_t)r * IN + c] = v;
        else
            t[r] = v;
    }
}

}  // namespace

// Network state owned by the context.
struct Mlp {
    bool ready = false;
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *W1 = nullptr, *W2 = nullptr, *W3 = nullptr, *W4 = nullptr, *W2t = nullptr, *W3t = nullptr,
             *W4t = nullptr;
    int64_t step = 0;
    // training scratch for minibatches of up to B records
    int B = 0;
    float *X = nullptr, *t = nullptr, *y = nullptr, *z = nullptr, *loss = nullptr;
    uint16_t *hfm = nullptr, *dzfm = nullptr, *dy = nullptr;
    uint32_t *perm = nullptr;
    int64_t perm_n = 0;
    Weights w() const { return Weights{W1, W2, W3, W4, W2t, W3t, W4t, p}; }
};

size_t mlp_forward_lds() { return sizeof(uint16_t) * (size_t)2 * 16 * S_H; }
size_t mlp_backward_lds() { return sizeof(uint16_t) * (size_t)4 * 2 * 16 * S_H; }

hipError_t mlp_predict(const Mlp &m, const float *X, int64_t n, const uint32_t *n_dev, float *y, int grid,
                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // one block per 16-record tile, up to 4,096 (then each block loops)
    const int g = grid > 0 ? grid : (int)std::min<int64_t>((n + 15) / 16, 4096);
    hipLaunchKernelGGL(k_forward, dim3(g), dim3(kThreads), mlp_forward_lds(), s, m.w(), X, n, n_dev, y,
                       Save{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0});
    return hipGetLastError();
}

}  // namespace gosma

namespace {

using gosma::Mlp;

template <class T>
hipError_t dalloc(T *&p, size_t n)
{
    return hipMalloc((void **)&p, sizeof(T) * std::max<size_t>(n, 1));
}
template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void free_scratch(Mlp *m)
{
    dfree(m->X);
    dfree(m->t);
    dfree(m->y);
    dfree(m->z);
    dfree(m->loss);
    dfree(m->hfm);
    dfree(m->dzfm);
    dfree(m->dy);
    m->B = 0;
}

hipError_t ensure_mlp(gosma_ctx *ctx)
{
    if (ctx->mlp) return hipSuccess;
    Mlp *m = new Mlp;
    hipError_t e;
    const int NP = GOSMA_MLP_PARAMS;
    if ((e = dalloc(m->p, NP)) || (e = dalloc(m->m, NP)) || (e = dalloc(m->v, NP)) || (e = dalloc(m->grad, NP)) ||
        (e = dalloc(m->W1, 128 * 32)) || (e = dalloc(m->W2, 128 * 128)) || (e = dalloc(m->W3, 128 * 128)) ||
        (e = dalloc(m->W4, 16 * 128)) || (e = dalloc(m->W2t, 128 * 128)) || (e = dalloc(m->W3t, 128 * 128)) ||
        (e = dalloc(m->W4t, 128 * 16))) {
        delete m;
        return e;
    }
    ctx->mlp = m;
    return hipSuccess;
}

hipError_t ensure_scratch(Mlp *m, int B)
{
    if (m->B >= B) return hipSuccess;
    free_scratch(m);
    hipError_t e;
    if ((e = dalloc(m->X, (size_t)B * 20)) || (e = dalloc(m->t, B)) || (e = dalloc(m->y, B)) ||
        (e = dalloc(m->z, (size_t)3 * B * 128)) || (e = dalloc(m->loss, 1)) ||
        (e = dalloc(m->hfm, (size_t)(32 + 3 * 128) * B)) || (e = dalloc(m->dzfm, (size_t)(16 + 3 * 128) * B)) ||
        (e = dalloc(m->dy, (size_t)16 * B)))
        return e;
    // unused rows of the padded output-layer operands stay zero
    if ((e = hipMemset(m->dzfm, 0, sizeof(uint16_t) * 16 * (size_t)B)) ||
        (e = hipMemset(m->dy, 0, sizeof(uint16_t) * 16 * (size_t)B)) ||
        (e = hipMemset(m->hfm, 0, sizeof(uint16_t) * (size_t)(32 + 3 * 128) * B)))
        return e;
    m->B = B;
    return hipSuccess;
}

hipError_t pack_weights(Mlp *m, hipStream_t s)
{
    hipLaunchKernelGGL(gosma::k_pack, dim3(64), dim3(256), 0, s, m->p, m->W1, m->W2, m->W3, m->W4, m->W2t, m->W3t,
                       m->W4t);
    m->ready = true;
    return hipGetLastError();
}

// One minibatch: forward (saving activations), loss, backward, weight
// gradients into m->grad.  X, t on device, n <= m->B (multiple of 16 padding
// is handled by the kernels).
hipError_t minibatch_grad(Mlp *m, const float *X, const float *t, int n, hipStream_t s)
{
    using namespace gosma;
    const int B = m->B;
    Save sv{m->z, m->z + (size_t)B * 128, m->z + (size_t)2 * B * 128, m->hfm, m->hfm + (size_t)32 * B,
            m->hfm + (size_t)(32 + 128) * B, m->hfm + (size_t)(32 + 256) * B, B};
    const int tiles = (n + 15) / 16;
    const int g = std::max(1, std::min(1024, (tiles + 3) / 4));
    hipLaunchKernelGGL(k_forward, dim3(std::max(1, std::min(4096, tiles))), dim3(kThreads), mlp_forward_lds(), s,
                       m->w(), X, (int64_t)n, (const uint32_t *)nullptr, m->y, sv);
    hipLaunchKernelGGL(k_loss, dim3(std::max(1, std::min(256, (B + 255) / 256))), dim3(256), 0, s, m->y, t, n, B,
                       m->dy, m->dzfm, m->loss);
    uint16_t *dz3 = m->dzfm + (size_t)16 * B, *dz2 = dz3 + (size_t)128 * B, *dz1 = dz2 + (size_t)128 * B;
    hipLaunchKernelGGL(k_backward, dim3(g), dim3(kThreads), mlp_backward_lds(), s, m->w(), m->dy, sv, dz3, dz2, dz1,
                       n);
    WgradJob j1{dz1, sv.h0fm, 128, IN, 2, oW1, ob1};
    WgradJob j2{dz2, sv.h1fm, 128, 128, 8, oW2, ob2};
    WgradJob j3{dz3, sv.h2fm, 128, 128, 8, oW3, ob3};
    WgradJob j4{m->dzfm, sv.h3fm, 1, 128, 8, oW4, ob4};
    const int ntiles = 16 + 64 + 64 + 8;
    // the K loop runs over padded records; rows beyond n are zero in both operands
    hipLaunchKernelGGL(k_wgrad, dim3((ntiles + 3) / 4), dim3(kThreads), 0, s, j1, j2, j3, j4, B, tiles * 16,
                       m->grad);
    return hipGetLastError();
}

}  // namespace

extern "C" {

void gosma_release_mlp(gosma_ctx *ctx)
{
    if (!ctx || !ctx->mlp) return;
    Mlp *m = ctx->mlp;
    free_scratch(m);
    dfree(m->p);
    dfree(m->m);
    dfree(m->v);
    dfree(m->grad);
    dfree(m->W1);
    dfree(m->W2);
    dfree(m->W3);
    dfree(m->W4);
    dfree(m->W2t);
    dfree(m->W3t);
    dfree(m->W4t);
    dfree(m->perm);
    delete m;
    ctx->mlp = nullptr;
}

int gosma_mlp_set_params(gosma_ctx *ctx, const float *params)
{
    if (!ctx || !params) return GOSMA_E_INVAL;
    ctx->err.clear();
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) || (e = ensure_mlp(ctx))) {
        ctx->err = std::string("gosma_mlp_set_params: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    Mlp *m = ctx->mlp;
    const size_t bytes = sizeof(float) * GOSMA_MLP_PARAMS;
    if ((e = hipMemcpy(m->p, params, bytes, hipMemcpyHostToDevice)) || (e = hipMemset(m->m, 0, bytes)) ||
        (e = hipMemset(m->v, 0, bytes)) || (e = pack_weights(m, nullptr)) || (e = hipDeviceSynchronize())) {
        ctx->err = std::string("gosma_mlp_set_params: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    m->step = 0;
    return GOSMA_OK;
}

int gosma_mlp_init(gosma_ctx *ctx, uint64_t seed)
{
    if (!ctx) return GOSMA_E_INVAL;
    // He initialisation of the weights, small biases (host RNG, deterministic per seed)
    std::vector<float> p(GOSMA_MLP_PARAMS);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> N01(0.0f, 1.0f);
    auto fill = [&](int off, int rows, int cols) {
        const float sd = std::sqrt(2.0f / (float)cols);
        for (int i = 0; i < rows * cols; ++i) p[off + i] = sd * N01(rng);
    };
    using namespace gosma;
    fill(oW1, 128, 20);
    fill(oW2, 128, 128);
    fill(oW3, 128, 128);
    fill(oW4, 1, 128);
    for (int off : {ob1, ob2, ob3}) std::fill(p.begin() + off, p.begin() + off + 128, 0.0f);
    p[ob4] = 0.0f;
    return gosma_mlp_set_params(ctx, p.data());
}

int gosma_mlp_get_params(gosma_ctx *ctx, float *params)
{
    if (!ctx || !params) return GOSMA_E_INVAL;
    if (!ctx->mlp || !ctx->mlp->ready) {
        ctx->err = "no network: call gosma_mlp_init or gosma_mlp_set_params";
        return GOSMA_E_STATE;
    }
    hipError_t e = hipMemcpy(params, ctx->mlp->p, sizeof(float) * GOSMA_MLP_PARAMS, hipMemcpyDeviceToHost);
    if (e) {
        ctx->err = std::string("gosma_mlp_get_params: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    return GOSMA_OK;
}

int gosma_mlp_predict(gosma_ctx *ctx, const float *x, int64_t n, float *y, void *stream)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!ctx->mlp || !ctx->mlp->ready) {
        ctx->err = "no network: call gosma_mlp_init or gosma_mlp_set_params";
        return GOSMA_E_STATE;
    }
    if (n < 0 || (n > 0 && (!x || !y))) {
        ctx->err = "invalid arguments";
        return GOSMA_E_INVAL;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (!e) e = gosma::mlp_predict(*ctx->mlp, x, n, nullptr, y, 0, (hipStream_t)stream);
    if (e) {
        ctx->err = std::string("gosma_mlp_predict: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    return GOSMA_OK;
}

int gosma_mlp_loss_grad(gosma_ctx *ctx, const float *records, int64_t n, double *loss, float *grad)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!ctx->mlp || !ctx->mlp->ready) {
        ctx->err = "no network: call gosma_mlp_init or gosma_mlp_set_params";
        return GOSMA_E_STATE;
    }
    if (n < 1 || n > (1 << 20) || !records || !loss || !grad) {
        ctx->err = "invalid arguments (1 <= n <= 2^20)";
        return GOSMA_E_INVAL;
    }
    Mlp *m = ctx->mlp;
    const int B = (int)((n + 15) / 16 * 16);
    hipError_t e;
    std::vector<uint32_t> perm(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    uint32_t *dperm = nullptr;
    float zero = 0.0f, hl = 0.0f;
    if ((e = hipSetDevice(ctx->device)) || (e = ensure_scratch(m, B)) || (e = dalloc(dperm, n)) ||
        (e = hipMemcpy(dperm, perm.data(), 4 * n, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(m->loss, &zero, 4, hipMemcpyHostToDevice))) {
        dfree(dperm);
        ctx->err = std::string("gosma_mlp_loss_grad: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    hipLaunchKernelGGL(gosma::k_gather, dim3(256), dim3(256), 0, nullptr, records, dperm, (int64_t)0, (int)n, m->X,
                       m->t);
    e = minibatch_grad(m, m->X, m->t, (int)n, nullptr);
    if (!e) e = hipMemcpy(grad, m->grad, sizeof(float) * GOSMA_MLP_PARAMS, hipMemcpyDeviceToHost);
    if (!e) e = hipMemcpy(&hl, m->loss, 4, hipMemcpyDeviceToHost);
    dfree(dperm);
    if (e) {
        ctx->err = std::string("gosma_mlp_loss_grad: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    *loss = (double)hl / (double)n;
    return GOSMA_OK;
}

int gosma_mlp_train(gosma_ctx *ctx, const float *records, int64_t n, int epochs, int batch, float lr, uint64_t seed,
                    float *loss_per_epoch)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!ctx->mlp || !ctx->mlp->ready) {
        ctx->err = "no network: call gosma_mlp_init or gosma_mlp_set_params";
        return GOSMA_E_STATE;
    }
    if (n < 1 || n > ((int64_t)1 << 31) || !records || epochs < 1 || batch < 16 || batch > 65536 ||
        !(lr > 0)) {
        ctx->err = "invalid arguments (n >= 1, epochs >= 1, 16 <= batch <= 65536, lr > 0)";
        return GOSMA_E_INVAL;
    }
    Mlp *m = ctx->mlp;
    const int B = (batch + 15) / 16 * 16;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) || (e = ensure_scratch(m, B))) {
        ctx->err = std::string("gosma_mlp_train: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    if (m->perm_n < n) {
        dfree(m->perm);
        if ((e = dalloc(m->perm, n))) {
            ctx->err = std::string("gosma_mlp_train: ") + hipGetErrorString(e);
            return GOSMA_E_NOMEM;
        }
        m->perm_n = n;
    }
    std::vector<uint32_t> perm(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    std::mt19937_64 rng(seed);
    const float b1 = 0.9f, b2 = 0.999f;
    for (int ep = 0; ep < epochs && !e; ++ep) {
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[rng() % (uint64_t)(i + 1)]);
        const float zero = 0.0f;
        if ((e = hipMemcpy(m->perm, perm.data(), 4 * (size_t)n, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(m->loss, &zero, 4, hipMemcpyHostToDevice)))
            break;
        for (int64_t off = 0; off < n && !e; off += B) {
            const int nb = (int)std::min<int64_t>(B, n - off);
            hipLaunchKernelGGL(gosma::k_gather, dim3(256), dim3(256), 0, nullptr, records, m->perm, off, nb, m->X,
                               m->t);
            e = minibatch_grad(m, m->X, m->t, nb, nullptr);
            if (e) break;
            // the loss gradient is the mean over this minibatch
            m->step += 1;
            const float c1 = 1.0f - std::pow(b1, (float)m->step), c2 = 1.0f - std::pow(b2, (float)m->step);
            hipLaunchKernelGGL(gosma::k_adam, dim3(64), dim3(256), 0, nullptr, m->p, m->grad, m->m, m->v,
                               GOSMA_MLP_PARAMS, lr, b1, b2, c1, c2, 1e-8f);
            e = pack_weights(m, nullptr);
        }
        float hl = 0.0f;
        if (!e) e = hipMemcpy(&hl, m->loss, 4, hipMemcpyDeviceToHost);
        if (!e && loss_per_epoch) loss_per_epoch[ep] = hl / (float)n;
    }
    if (e) {
        ctx->err = std::string("gosma_mlp_train: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    return GOSMA_OK;
}

}  // extern "C"

bool gosma_ctx::mlp_ready() const { return mlp && mlp->ready; }
