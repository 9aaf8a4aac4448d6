// Learned importance sampling for VSamp: per-vertex features and a small MLP
// (8 -> 64 -> 64 -> 1, ReLU) with BF16 weights and FP32 accumulation on the
// matrix cores, trained on exact per-vertex counts (log1p B_v) with Adam.
// The network only chooses sampling probabilities for bfc_vsamp; it never
// changes a count.
//
// MFMA formulation.  v_mfma_f32_16x16x16_bf16 multiplies a 16x16 A tile by a
// 16x16 B tile (wave64; lane l = 16 g + c holds A[c][4g..4g+3],
// B[4g..4g+3][c] and D[4g..4g+3][c]).  The layers are computed transposed,
// H^T = W^T X^T, with 16 rows of the batch per tile: then a layer's output
// tile is, lane for lane, the B operand of the next layer, and the backward
// activation product dH1^T = W2 dZ2^T needs no data movement either.  The
// weight gradients reduce over the batch (K = rows) and take their operands
// through a wave-private LDS transpose.
#include "common.h"

namespace bfc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Parameter layout (float offsets) of the FP32 master copy, the Adam moments
// and the gradients; the BF16 copy holds W1, W2, w3 at the same offsets.
constexpr int P_W1 = 0;        // [8][64]  input feature x hidden 1
constexpr int P_B1 = 512;      // [64]
constexpr int P_W2 = 576;      // [64][64] hidden 1 x hidden 2
constexpr int P_B2 = 4672;     // [64]
constexpr int P_W3 = 4736;     // [64]
constexpr int P_B3 = 4800;     // [1]
constexpr int P_N = 4801;
constexpr int NFEAT = 8;

__device__ inline uint16_t f2bf(float f) {      // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 v;
    v[0] = (short)f2bf(a);
    v[1] = (short)f2bf(b);
    v[2] = (short)f2bf(c);
    v[3] = (short)f2bf(d);
    return v;
}

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ features
// Per vertex v with neighbours u: side, log1p d_v, log1p sum d_u, log1p sum
// d_u^2, log1p max d_u, log1p sum (d_u - 1) (paths v-u-w, w != v), log1p
// C(d_v, 2), log1p(sum d_u / d_v); each log term scaled by 1/8.  Rows by
// global id (L ids, then n_left + R id), BF16.
// A group of NFEAT lanes per vertex (most vertices have few neighbours, so
// a wave per vertex left most lanes idle): the group sums its neighbours'
// degrees, reduces over its lanes, and lane i writes feature i.  The sums
// are integers below 2^53, exact in binary64 in any order.
constexpr uint32_t FGROUP = NFEAT;
__global__ __launch_bounds__(256) void k_features(const uint32_t *offS, const uint32_t *adjS,
                                                  const uint32_t *offT, const uint32_t *idS,
                                                  uint32_t nS, uint32_t row0, float side,
                                                  uint16_t *feat) {
    const uint32_t lane = threadIdx.x & (FGROUP - 1), gpb = blockDim.x / FGROUP;
    for (uint32_t v = blockIdx.x * gpb + threadIdx.x / FGROUP; v < nS; v += gridDim.x * gpb) {
        const uint32_t b = offS[v], e = offS[v + 1];
        double s1 = 0, s2 = 0, s3 = 0;
        uint32_t mx = 0;
        for (uint32_t k = b + lane; k < e; k += FGROUP) {
            const uint32_t u = adjS[k];
            const double d = (double)(offT[u + 1] - offT[u]);
            s1 += d;
            s2 += d * d;
            s3 += d - 1.0;
            mx = max(mx, (uint32_t)d);
        }
        // partners lane ^ o (o < FGROUP) are in the same group
#pragma unroll
        for (int o = FGROUP / 2; o > 0; o >>= 1) {
            s1 += __shfl_xor(s1, o, WAVE);
            s2 += __shfl_xor(s2, o, WAVE);
            s3 += __shfl_xor(s3, o, WAVE);
            mx = max(mx, (uint32_t)__shfl_xor(mx, o, WAVE));
        }
        {
            const double dv = (double)(e - b);
            double x;
            switch (lane) {
                case 0: x = 8.0 * side; break;
                case 1: x = log1p(dv); break;
                case 2: x = log1p(s1); break;
                case 3: x = log1p(s2); break;
                case 4: x = log1p((double)mx); break;
                case 5: x = log1p(s3); break;
                case 6: x = log1p(dv > 1.0 ? dv * (dv - 1.0) * 0.5 : 0.0); break;
                default: x = log1p(dv > 0 ? s1 / dv : 0.0); break;
            }
            feat[(uint64_t)(row0 + idS[v]) * NFEAT + lane] = f2bf((float)(x * 0.125));
        }
    }
}

// ------------------------------------------------------------------ network tiles
struct MlpArgs {
    const uint16_t *X;       // rows x 8 BF16 (or more rows, gathered through idx)
    const uint32_t *idx;     // training: row r of the batch is X row idx[r]; null = r
    const float *target;     // indexed like X (training) or null
    float *y;                // rows (inference) or null
    uint32_t rows;
    const float *prm;        // FP32 parameters (biases read from here)
    const uint16_t *wbf;     // BF16 W1, W2, w3
    float *part;             // training: per-wave partial sums, GSTRIDE floats per wave
    float inv_rows;          // 1 / rows of the mini-batch (training)
};

struct Weights {
    bf16x4 a1[4];            // layer 1 A tiles: W1^T[16t + c][4g + i]
    bf16x4 a2[4][4];         // layer 2 A tiles [t2][t]: W2^T[16 t2 + c][16 t + 4g + i]
    float b1[4][4], b2[4][4], w3[4][4], b3;   // per lane: feature 16t + 4g + i
};

__device__ inline void load_weights(const MlpArgs &a, Weights &w) {
    const uint32_t l = threadIdx.x & (WAVE - 1), g = l >> 4, c = l & 15;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        bf16x4 v;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t k = 4 * g + i;           // input feature (padded to 16)
            v[i] = k < NFEAT ? (short)a.wbf[P_W1 + k * 64 + 16 * t + c] : (short)0;
        }
        w.a1[t] = v;
#pragma unroll
        for (int t2 = 0; t2 < 4; t2++) {
#pragma unroll
            for (int i = 0; i < 4; i++)
                v[i] = (short)a.wbf[P_W2 + (16 * t + 4 * g + i) * 64 + 16 * t2 + c];
            w.a2[t2][t] = v;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t f = 16 * t + 4 * g + i;
            w.b1[t][i] = a.prm[P_B1 + f];
            w.b2[t][i] = a.prm[P_B2 + f];
            w.w3[t][i] = bf2f(a.wbf[P_W3 + f]);
        }
    }
    w.b3 = a.prm[P_B3];
}

// Forward of one 16-row tile: Z1^T, H1^T (BF16 B operands), Z2^T, H2^T and
// y[row c] on every lane of that row.
struct Acts {
    bf16x4 x;                // layer 1 B operand: X[row c][4g..4g+3]
    f32x4 z1[4], z2[4];
    bf16x4 h1[4];
    float h2[4][4];
    float y;
};

__device__ inline void forward_tile(const MlpArgs &a, const Weights &w, uint32_t row0, Acts &s) {
    const uint32_t l = threadIdx.x & (WAVE - 1), g = l >> 4, c = l & 15;
    const uint32_t row = row0 + c;
    bf16x4 x = {0, 0, 0, 0};
    if (g < 2 && row < a.rows) {
        const uint64_t src = a.idx ? a.idx[row] : row;
        const uint2 raw = *(const uint2 *)(a.X + src * NFEAT + 4 * g);
        x[0] = (short)(raw.x & 0xFFFF);
        x[1] = (short)(raw.x >> 16);
        x[2] = (short)(raw.y & 0xFFFF);
        x[3] = (short)(raw.y >> 16);
    }
    s.x = x;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const f32x4 zero = {0, 0, 0, 0};
        f32x4 z = mfma(w.a1[t], x, zero);
#pragma unroll
        for (int i = 0; i < 4; i++) z[i] += w.b1[t][i];
        s.z1[t] = z;
        s.h1[t] = pack4(fmaxf(z[0], 0.f), fmaxf(z[1], 0.f), fmaxf(z[2], 0.f), fmaxf(z[3], 0.f));
    }
    float part = 0.f;
#pragma unroll
    for (int t2 = 0; t2 < 4; t2++) {
        f32x4 z = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; t++) z = mfma(w.a2[t2][t], s.h1[t], z);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            z[i] += w.b2[t2][i];
            s.h2[t2][i] = fmaxf(z[i], 0.f);
            part += s.h2[t2][i] * w.w3[t2][i];
        }
        s.z2[t2] = z;
    }
    part += __shfl_xor(part, 16, WAVE);
    part += __shfl_xor(part, 32, WAVE);
    s.y = part + w.b3;
}

__global__ __launch_bounds__(256) void k_mlp_forward(MlpArgs a) {
    Weights w;
    load_weights(a, w);
    const uint32_t l = threadIdx.x & (WAVE - 1);
    const uint32_t wave = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const uint32_t nwaves = gridDim.x * (blockDim.x / WAVE);
    for (uint32_t row0 = wave * 16; row0 < a.rows; row0 += nwaves * 16) {
        Acts s;
        forward_tile(a, w, row0, s);
        if (l < 16 && row0 + l < a.rows) a.y[row0 + l] = s.y;
    }
}

// Wave-private 16x16 BF16 tile in LDS: written from the D layout
// (lane 16g + c holds [4g+i][c]) and read back as an operand in which lane
// 16g + c needs [c][4g..4g+3] (the transpose).
__device__ inline void tile_put(uint16_t *t, const float v[4]) {
    const uint32_t l = threadIdx.x & (WAVE - 1), g = l >> 4, c = l & 15;
#pragma unroll
    for (int i = 0; i < 4; i++) t[(4 * g + i) * 16 + c] = f2bf(v[i]);
}

__device__ inline bf16x4 tile_get_t(const uint16_t *t) {
    const uint32_t l = threadIdx.x & (WAVE - 1), g = l >> 4, c = l & 15;
    const uint2 raw = *(const uint2 *)(t + c * 16 + 4 * g);
    bf16x4 v;
    v[0] = (short)(raw.x & 0xFFFF);
    v[1] = (short)(raw.x >> 16);
    v[2] = (short)(raw.y & 0xFFFF);
    v[3] = (short)(raw.y >> 16);
    return v;
}

__device__ inline void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

constexpr int MLP_WAVES = 4;
constexpr int MLP_MAX_WAVES = 1024;   // one wave per SIMD at this kernel's register use
constexpr int GSTRIDE = 4864;         // partial row: P_N gradients, then the loss

// Forward and backward of the mean squared error of y against the target
// over tiles of 16 rows; each wave accumulates its tiles in registers and
// writes one partial row (every gradient and its squared-error sum) that
// k_grad_reduce sums over the waves in a fixed order.
__global__ __launch_bounds__(MLP_WAVES * WAVE) void k_mlp_grad(MlpArgs a) {
    __shared__ uint16_t tiles[MLP_WAVES][13][256];
    Weights w;
    load_weights(a, w);
    const uint32_t l = threadIdx.x & (WAVE - 1), g = l >> 4, c = l & 15;
    const uint32_t wv = threadIdx.x / WAVE;
    uint16_t *tX = tiles[wv][12];             // tiles 0-3 H1^T, 4-7 dZ2^T, 8-11 dZ1^T
    // W2 tiles of the backward product dH1^T = W2 dZ2^T: [t1][t2] = W2[16 t1 + c][16 t2 + 4g + i]
    bf16x4 a2b[4][4];
#pragma unroll
    for (int t1 = 0; t1 < 4; t1++)
#pragma unroll
        for (int t2 = 0; t2 < 4; t2++)
#pragma unroll
            for (int i = 0; i < 4; i++)
                a2b[t1][t2][i] = (short)a.wbf[P_W2 + (16 * t1 + c) * 64 + 16 * t2 + 4 * g + i];
    f32x4 gW2[4][4], gW1[4];
    float gb1[4][4], gb2[4][4], gw3[4][4], gb3 = 0.f, loss = 0.f;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        gW1[t] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < 4; u++) gW2[t][u] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 4; i++) gb1[t][i] = gb2[t][i] = gw3[t][i] = 0.f;
    }
    const uint32_t wave = blockIdx.x * MLP_WAVES + wv;
    const uint32_t nwaves = gridDim.x * MLP_WAVES;
    for (uint32_t row0 = wave * 16; row0 < a.rows; row0 += nwaves * 16) {
        Acts s;
        forward_tile(a, w, row0, s);
        const uint32_t row = row0 + c;
        const bool valid = row < a.rows;
        const float err = valid ? s.y - a.target[a.idx ? a.idx[row] : row] : 0.f;
        const float dy = 2.f * err * a.inv_rows;
        if (g == 0) {
            loss += err * err;
            gb3 += dy;
        }
        // dZ2^T = relu'(Z2) * w3 * dy
        bf16x4 dz2[4];
#pragma unroll
        for (int t2 = 0; t2 < 4; t2++) {
            float d[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                d[i] = s.z2[t2][i] > 0.f ? w.w3[t2][i] * dy : 0.f;
                gb2[t2][i] += d[i];
                gw3[t2][i] += s.h2[t2][i] * dy;
            }
            dz2[t2] = pack4(d[0], d[1], d[2], d[3]);
            tile_put(tiles[wv][4 + t2], d);
        }
        // dH1^T = W2 dZ2^T, dZ1^T = relu'(Z1) dH1^T
        float dz1[4][4];
#pragma unroll
        for (int t1 = 0; t1 < 4; t1++) {
            f32x4 d = {0, 0, 0, 0};
#pragma unroll
            for (int t2 = 0; t2 < 4; t2++) d = mfma(a2b[t1][t2], dz2[t2], d);
#pragma unroll
            for (int i = 0; i < 4; i++) {
                dz1[t1][i] = s.z1[t1][i] > 0.f ? d[i] : 0.f;
                gb1[t1][i] += dz1[t1][i];
            }
            tile_put(tiles[wv][8 + t1], dz1[t1]);
            float h[4];
#pragma unroll
            for (int i = 0; i < 4; i++) h[i] = bf2f((uint16_t)s.h1[t1][i]);
            tile_put(tiles[wv][t1], h);
        }
        // X tile as [feature][row] for the dW1 operand
        {
            float xv[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; i++) xv[i] = bf2f((uint16_t)s.x[i]);
            // lane (g, c) holds X[row c][4g + i]: store as [4g + i][c]
            tile_put(tX, xv);
        }
        wave_fence();
        // dW2[f1][f2] += sum_rows H1[row][f1] dZ2[row][f2]: A = H1 (rows as k), B = dZ2
        bf16x4 hA[4], zB[4], z1B[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            hA[t] = tile_get_t(tiles[wv][t]);
            zB[t] = tile_get_t(tiles[wv][4 + t]);
            z1B[t] = tile_get_t(tiles[wv][8 + t]);
        }
        const bf16x4 xA = tile_get_t(tX);
#pragma unroll
        for (int t1 = 0; t1 < 4; t1++)
#pragma unroll
            for (int t2 = 0; t2 < 4; t2++) gW2[t1][t2] = mfma(hA[t1], zB[t2], gW2[t1][t2]);
        // dW1[k][f1] += sum_rows X[row][k] dZ1[row][f1]
#pragma unroll
        for (int t1 = 0; t1 < 4; t1++) gW1[t1] = mfma(xA, z1B[t1], gW1[t1]);
        wave_fence();
    }
    // per-feature sums over the 16 rows (lanes c) of each lane group g
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                gb1[t][i] += __shfl_xor(gb1[t][i], o, WAVE);
                gb2[t][i] += __shfl_xor(gb2[t][i], o, WAVE);
                gw3[t][i] += __shfl_xor(gw3[t][i], o, WAVE);
            }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        gb3 += __shfl_xor(gb3, o, WAVE);
        loss += __shfl_xor(loss, o, WAVE);
    }
    float *part = a.part + (uint64_t)wave * GSTRIDE;
#pragma unroll
    for (int t1 = 0; t1 < 4; t1++) {
#pragma unroll
        for (int t2 = 0; t2 < 4; t2++)
#pragma unroll
            for (int i = 0; i < 4; i++)
                part[P_W2 + (16 * t1 + 4 * g + i) * 64 + 16 * t2 + c] = gW2[t1][t2][i];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t k = 4 * g + i;
            if (k < NFEAT) part[P_W1 + k * 64 + 16 * t1 + c] = gW1[t1][i];
        }
        if (c == 0) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const uint32_t f = 16 * t1 + 4 * g + i;
                part[P_B1 + f] = gb1[t1][i];
                part[P_B2 + f] = gb2[t1][i];
                part[P_W3 + f] = gw3[t1][i];
            }
        }
    }
    if (l == 0) {
        part[P_B3] = gb3;
        part[P_N] = loss;
    }
}

// grad[j] (and *loss for j = P_N) = sum over the waves of the partial rows,
// in a fixed order: the 16 waves of a block each sum a contiguous sixteenth
// of the rows for 64 columns, then the sixteen partial sums are added in
// wave order.
constexpr int RED_WAVES = 16;

__global__ __launch_bounds__(RED_WAVES * WAVE) void k_grad_reduce(const float *part, uint32_t nw,
                                                                  float *grad, float *loss) {
    __shared__ float q[RED_WAVES][WAVE];
    const uint32_t lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const uint32_t j = blockIdx.x * WAVE + lane;
    const uint32_t per = (nw + RED_WAVES - 1) / RED_WAVES, w0 = wv * per,
                   w1 = min(nw, w0 + per);
    float s = 0.f;
    if (j <= (uint32_t)P_N)
        for (uint32_t w = w0; w < w1; w++) s += part[(uint64_t)w * GSTRIDE + j];
    q[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && j <= (uint32_t)P_N) {
        float t = q[0][lane];
#pragma unroll
        for (int i = 1; i < RED_WAVES; i++) t += q[i][lane];
        if (j < (uint32_t)P_N) grad[j] = t; else *loss = t;
    }
}

// Adam on the FP32 master copy, then refresh the BF16 weights.
__global__ void k_adam(float *prm, float *m1, float *m2, const float *grad, uint16_t *wbf,
                       float lr, float beta1, float beta2, float eps, float corr1, float corr2) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < (uint32_t)P_N;
         j += gridDim.x * blockDim.x) {
        const float gr = grad[j];
        const float a = beta1 * m1[j] + (1.f - beta1) * gr;
        const float b = beta2 * m2[j] + (1.f - beta2) * gr * gr;
        m1[j] = a;
        m2[j] = b;
        const float p = prm[j] - lr * (a / corr1) / (sqrtf(b / corr2) + eps);
        prm[j] = p;
        wbf[j] = f2bf(p);
    }
}

__global__ void k_to_bf16(const float *prm, uint16_t *wbf) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < (uint32_t)P_N;
         j += gridDim.x * blockDim.x)
        wbf[j] = f2bf(prm[j]);
}

// Training targets log1p(B_v) / 8 from exact per-vertex counts.
__global__ void k_targets(const uint64_t *cnt, uint64_t n, float *t) {
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n;
         j += (uint64_t)gridDim.x * blockDim.x)
        t[j] = (float)(log1p((double)cnt[j]) * 0.125);
}

// Sampling probabilities from predictions of log1p(B_v)/8: q_v =
// max(expm1(8 y_v), floor * mean) with mean the mean of the positive
// predicted counts and floor > 0, so every q_v > 0 (the Hansen-Hurwitz
// estimate stays unbiased whatever the network predicts); when no prediction
// is positive (mean 0) every q_v = 1, plain uniform sampling.  The mean is
// reduced in a fixed order (per-block partials, then the partials in block
// order), so the probabilities are reproducible.
constexpr int PROB_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_pred_partial(const float *y, uint64_t n, double *part) {
    __shared__ double red[256 / WAVE];
    const uint64_t chunk = (n + PROB_BLOCKS - 1) / PROB_BLOCKS;
    const uint64_t b = blockIdx.x * chunk, e = min(n, b + chunk);
    double s = 0;
    for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        const double v = expm1(8.0 * (double)y[i]);
        s += v > 0 ? v : 0.0;
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < 256 / WAVE; w++) t += red[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(256) void k_pred_probs(const float *y, uint64_t n, double floor_frac,
                                                    const double *part, double *probs,
                                                    double *mean_out) {
    __shared__ double mean_s;
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < PROB_BLOCKS; i++) t += part[i];
        mean_s = t / (double)n;
        if (blockIdx.x == 0 && mean_out) *mean_out = mean_s;
    }
    __syncthreads();
    const double fl = floor_frac * mean_s;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double v = expm1(8.0 * (double)y[i]);
        probs[i] = mean_s > 0.0 ? (v > fl ? v : fl) : 1.0;
    }
}

static inline unsigned grid_for(uint64_t n, int nt = 256) {
    uint64_t g = (n + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > 65535ull * 16) g = 65535ull * 16;
    return (unsigned)g;
}

}  // namespace bfc

using namespace bfc;

extern "C" {

int bfc_mlp_param_count(void) { return P_N; }

int bfc_features(const bfc_graph *g, uint16_t *d_feat, hipStream_t s) {
    if (!g || !d_feat) return BFC_E_NULL;
    unsigned gl = grid_for(g->n_left, 256 / FGROUP), gr = grid_for(g->n_right, 256 / FGROUP);
    if (gl > 8192) gl = 8192;
    if (gr > 8192) gr = 8192;
    if (g->n_left)
        k_features<<<gl, 256, 0, s>>>(g->off_l, g->adj_l, g->off_r, g->id_l, g->n_left, 0, 0.f,
                                      d_feat);
    if (g->n_right)
        k_features<<<gr, 256, 0, s>>>(g->off_r, g->adj_r, g->off_l, g->id_r, g->n_right,
                                      g->n_left, 1.f, d_feat);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_mlp_bf16(const float *d_params, uint16_t *d_wbf16, hipStream_t s) {
    if (!d_params || !d_wbf16) return BFC_E_NULL;
    k_to_bf16<<<grid_for(P_N), 256, 0, s>>>(d_params, d_wbf16);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_mlp_forward(const uint16_t *d_x, uint32_t rows, const float *d_params,
                    const uint16_t *d_wbf16, float *d_y, hipStream_t s) {
    if (!d_x || !d_params || !d_wbf16 || !d_y) return BFC_E_NULL;
    if (rows == 0) return BFC_OK;
    MlpArgs a = {};
    a.X = d_x; a.rows = rows; a.prm = d_params; a.wbf = d_wbf16; a.y = d_y;
    unsigned grid = grid_for((uint64_t)(rows + 15) / 16, 4);
    if (grid > 4096) grid = 4096;
    k_mlp_forward<<<grid, 256, 0, s>>>(a);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_mlp_targets(const uint64_t *d_counts, uint64_t n, float *d_target, hipStream_t s) {
    if (!d_counts || !d_target) return BFC_E_NULL;
    if (n == 0) return BFC_OK;
    unsigned grid = grid_for(n);
    if (grid > 8192) grid = 8192;
    k_targets<<<grid, 256, 0, s>>>(d_counts, n, d_target);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

static uint32_t grad_blocks(uint32_t rows) {
    uint64_t b = ((uint64_t)rows + 16 * MLP_WAVES - 1) / (16 * MLP_WAVES);
    if (b < 1) b = 1;
    if (b > MLP_MAX_WAVES / MLP_WAVES) b = MLP_MAX_WAVES / MLP_WAVES;
    return (uint32_t)b;
}

int bfc_mlp_grad_ws_size(uint32_t rows, size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    *bytes = (size_t)grad_blocks(rows) * MLP_WAVES * GSTRIDE * sizeof(float);
    return BFC_OK;
}

int bfc_mlp_grad(const uint16_t *d_x, const float *d_target, const uint32_t *d_idx,
                 uint32_t rows, const float *d_params, const uint16_t *d_wbf16, float *d_grad,
                 float *d_loss, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!d_x || !d_target || !d_params || !d_wbf16 || !d_grad || !d_loss || !d_ws)
        return BFC_E_NULL;
    if (rows == 0) return BFC_E_ARG;
    const uint32_t blocks = grad_blocks(rows), nw = blocks * MLP_WAVES;
    if (ws_bytes < (size_t)nw * GSTRIDE * sizeof(float)) return BFC_E_WS_SMALL;
    MlpArgs a = {};
    a.X = d_x; a.idx = d_idx; a.target = d_target; a.rows = rows; a.prm = d_params;
    a.wbf = d_wbf16; a.part = (float *)d_ws; a.inv_rows = 1.f / (float)rows;
    k_mlp_grad<<<blocks, MLP_WAVES * WAVE, 0, s>>>(a);
    k_grad_reduce<<<(P_N + 1 + WAVE - 1) / WAVE, RED_WAVES * WAVE, 0, s>>>(a.part, nw, d_grad,
                                                                         d_loss);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_adam_step(float *d_params, float *d_m1, float *d_m2, const float *d_grad,
                  uint16_t *d_wbf16, float lr, float beta1, float beta2, float eps, uint32_t step,
                  hipStream_t s) {
    if (!d_params || !d_m1 || !d_m2 || !d_grad || !d_wbf16) return BFC_E_NULL;
    if (step == 0 || !(lr > 0.f)) return BFC_E_ARG;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    k_adam<<<grid_for(P_N), 256, 0, s>>>(d_params, d_m1, d_m2, d_grad, d_wbf16, lr, beta1, beta2,
                                         eps, c1, c2);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_probs_ws_size(size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    *bytes = PROB_BLOCKS * sizeof(double);
    return BFC_OK;
}

int bfc_probs_from_predictions(const float *d_y, uint64_t n, double floor_frac, double *d_probs,
                               double *d_mean, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!d_y || !d_probs || !d_ws) return BFC_E_NULL;
    if (n == 0 || !(floor_frac > 0.0) || !(floor_frac <= 1e300)) return BFC_E_ARG;
    if (ws_bytes < PROB_BLOCKS * sizeof(double)) return BFC_E_WS_SMALL;
    double *part = (double *)d_ws;
    k_pred_partial<<<PROB_BLOCKS, 256, 0, s>>>(d_y, n, part);
    unsigned grid = grid_for(n);
    if (grid > 8192) grid = 8192;
    k_pred_probs<<<grid, 256, 0, s>>>(d_y, n, floor_frac, part, d_probs, d_mean);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // extern "C"
