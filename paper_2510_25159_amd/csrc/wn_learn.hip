// Learned depth predictor (gfx950): per-pair features, an MLP
// 16 -> 64 -> 64 -> 1 (ReLU, BF16 weights, FP32 accumulation) trained by
// hand-written forward / backward / AdamW kernels on depths the near pass
// records, and a counting sort of the near queue into depth bins.
//
// The MLP's weights are read with wave-uniform addresses, so they reach the
// FMAs as scalar operands (no LDS traffic); one lane evaluates one pair.
#include "wn_device.h"
#include "wn_learn.h"

namespace wn {

// ---------------------------------------------------------------------------
// BF16 rounding (round to nearest even), kept in FP32 registers
// ---------------------------------------------------------------------------
__host__ __device__ inline float bf16_round(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

// The BF16 value of x (round to nearest even) as its 16-bit pattern.
__host__ __device__ inline uint16_t bf16_bits(float x) {
    const float r = bf16_round(x);
    uint32_t u;
    memcpy(&u, &r, 4);
    return (uint16_t)(u >> 16);
}

// Hidden unit that element e of lane group g's layer-2 operand takes in K
// step ks on the matrix cores (the order of the layer-1 accumulators; see
// the matrix-core inference below).
__host__ __device__ constexpr int l2_unit(int ks, int g, int e) { return 16 * (2 * ks + e / 4) + 4 * g + e % 4; }

// Fragment slot of parameter p in the BF16 fragment-order copy, or -1 (the
// biases and w3 are read as FP32).  Layer-1 tile t, lane i + 16 g, element e
// holds W1[16 t + i][8 g + e] (g < 2); layer-2 tile t, K step ks holds
// W2[16 t + i][l2_unit(ks, g, e)].
__host__ __device__ inline int frag_slot(int p) {
    if (p < kOffB1) {
        const int r = p / kMlpIn, k = p % kMlpIn;
        return ((r / 16) * 64 + r % 16 + 16 * (k / 8)) * 8 + k % 8;
    }
    if (p >= kOffW2 && p < kOffB2) {
        const int r = (p - kOffW2) / kMlpH, u = (p - kOffW2) % kMlpH;
        const int ks = (u / 16) / 2, g = (u % 16) / 4, e = 4 * ((u / 16) % 2) + u % 4;
        return 4 * 64 * 8 + (((r / 16) * 2 + ks) * 64 + r % 16 + 16 * g) * 8 + e;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// features of one (query, segment) pair (raw, unstandardised)
// ---------------------------------------------------------------------------
__device__ inline void pair_features(const Segs& sg, uint32_t s, double qx, double qy, double eps, float* f) {
    const double x0 = sg.p0x[s], y0 = sg.p0y[s], x1 = sg.pnx[s], y1 = sg.pny[s];
    const double B = sg.B[s];
    const double cx = 0.5 * (x0 + x1), cy = 0.5 * (y0 + y1);
    const double L = hypot(x1 - x0, y1 - y0);
    const double ux = L > 0.0 ? (x1 - x0) / L : 1.0, uy = L > 0.0 ? (y1 - y0) / L : 0.0;
    const double rx = qx - cx, ry = qy - cy;
    const double a = 0.5 * B, cf = 0.5 * L;
    const double bsemi = sqrt(fmax(a * a - cf * cf, 0.0));
    const double e1 = rx * ux + ry * uy, e2 = -rx * uy + ry * ux;
    const double d1 = hypot(qx - x0, qy - y0), d2 = hypot(qx - x1, qy - y1);
    const double* bx = sg.box + 4 * (size_t)s;
    const double dx = qx < bx[0] ? bx[0] - qx : (qx > bx[1] ? qx - bx[1] : 0.0);
    const double dy = qy < bx[2] ? bx[2] - qy : (qy > bx[3] ? qy - bx[3] : 0.0);
    const double dbox = sqrt(dx * dx + dy * dy);
    const double ainv = a > 0.0 ? 1.0 / a : 0.0;
    f[0] = (float)(e1 * ainv);
    f[1] = (float)(e2 * ainv);
    f[2] = (float)a;
    f[3] = (float)bsemi;
    f[4] = (float)sg.deg[s];
    f[5] = sg.wrange[2 * (size_t)s];
    f[6] = sg.wrange[2 * (size_t)s + 1];
    f[7] = (float)L;
    f[8] = (float)dbox;
    f[9] = (float)d1;
    f[10] = (float)d2;
    f[11] = (float)(B > 0.0 ? (d1 + d2) / B : 0.0);
    f[12] = (float)(B > 0.0 ? log2(B / fmax(eps, dbox)) : 0.0);
    f[13] = (float)B;
    f[14] = (float)cf;
    f[15] = e2 >= 0.0 ? 1.f : -1.f;
}


// ---------------------------------------------------------------------------
// MLP forward on standardised inputs; w = BF16-rounded parameters (FP32).
// ---------------------------------------------------------------------------
__device__ inline float mlp_forward(const float* __restrict__ w, const float* x, float* h1) {
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) {
        float acc = w[kOffB1 + i];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) acc = fmaf(w[kOffW1 + i * kMlpIn + k], x[k], acc);
        h1[i] = fmaxf(acc, 0.f);
    }
    float y = w[kOffB3];
    for (int j = 0; j < kMlpH; ++j) {
        float acc = w[kOffB2 + j];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) acc = fmaf(w[kOffW2 + j * kMlpH + i], h1[i], acc);
        y = fmaf(w[kOffW3 + j], fmaxf(acc, 0.f), y);
    }
    return y;
}

__device__ inline void standardise(float* f, const float* __restrict__ norm) {
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) f[k] = (f[k] - norm[k]) / norm[kMlpIn + k];
}

// ---------------------------------------------------------------------------
// feature kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pair_features(Segs sg, Points pts, const int32_t* pp, const int32_t* ps,
                                                       int64_t n, double eps, float* out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t q = pp[i];
    float f[kMlpIn];
    pair_features(sg, (uint32_t)ps[i], pts.u[q * pts.stride], pts.v[q * pts.stride], eps, f);
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) out[i * kMlpIn + k] = f[k];
}

__device__ inline void queue_query(const Points& pts, const NearQueue& nq, const uint8_t* seg_per, uint64_t i,
                                   uint32_t& s, double& qx, double& qy) {
    const uint2 e = nq.qs[i];
    s = e.y;
    qx = pts.u[(int64_t)e.x * pts.stride];
    qy = pts.v[(int64_t)e.x * pts.stride];
    if (nq.shift && seg_per[s]) {
        const double2 sh = nq.shift[i];
        qx -= sh.x;
        qy -= sh.y;
    }
}

__global__ __launch_bounds__(256) void k_queue_features(Segs sg, Points pts, NearQueue nq, const uint8_t* seg_per,
                                                        double eps, uint64_t limit, float* out) {
    unsigned long long n = *nq.count;
    n = n < nq.cap ? n : nq.cap;
    n = n < limit ? n : limit;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        uint32_t s;
        double qx, qy;
        queue_query(pts, nq, seg_per, i, s, qx, qy);
        float f[kMlpIn];
        pair_features(sg, s, qx, qy, eps, f);
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) out[i * kMlpIn + k] = f[k];
    }
}

__global__ __launch_bounds__(256) void k_predict(const float* __restrict__ w, const float* X, int64_t n, float* out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float x[kMlpIn], h1[kMlpH];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) x[k] = X[i * kMlpIn + k];
    out[i] = mlp_forward(w, x, h1);
}

// ---------------------------------------------------------------------------
// training: forward + per-sample backward, gradient reduction, AdamW
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fwd_bwd(const float* __restrict__ w, const float* X, const float* Y,
                                                 const int32_t* idx, int B, float delta, float* H1, float* H2,
                                                 float* DH1, float* DH2, float* DY, float* loss_acc) {
    __shared__ float s_loss[256];
    const int b = blockIdx.x * 256 + threadIdx.x;
    float loss = 0.f;
    if (b < B) {
        const int64_t j = idx[b];
        float x[kMlpIn], h1[kMlpH], dh1[kMlpH];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) x[k] = X[j * kMlpIn + k];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) {
            float acc = w[kOffB1 + i];
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k) acc = fmaf(w[kOffW1 + i * kMlpIn + k], x[k], acc);
            h1[i] = fmaxf(acc, 0.f);
            dh1[i] = 0.f;
        }
        float y = w[kOffB3];
        for (int jj = 0; jj < kMlpH; ++jj) {
            float acc = w[kOffB2 + jj];
#pragma unroll
            for (int i = 0; i < kMlpH; ++i) acc = fmaf(w[kOffW2 + jj * kMlpH + i], h1[i], acc);
            const float h2 = fmaxf(acc, 0.f);
            H2[(int64_t)b * kMlpH + jj] = h2;
            y = fmaf(w[kOffW3 + jj], h2, y);
        }
        const float r = y - Y[j];
        const float ar = fabsf(r);
        loss = ar <= delta ? 0.5f * r * r : delta * (ar - 0.5f * delta);
        const float g = (ar <= delta ? r : copysignf(delta, r)) / (float)B;
        DY[b] = g;
        for (int jj = 0; jj < kMlpH; ++jj) {
            const float h2 = H2[(int64_t)b * kMlpH + jj];
            const float d2 = h2 > 0.f ? g * w[kOffW3 + jj] : 0.f;
            DH2[(int64_t)b * kMlpH + jj] = d2;
#pragma unroll
            for (int i = 0; i < kMlpH; ++i) dh1[i] = fmaf(d2, w[kOffW2 + jj * kMlpH + i], dh1[i]);
        }
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) {
            H1[(int64_t)b * kMlpH + i] = h1[i];
            DH1[(int64_t)b * kMlpH + i] = h1[i] > 0.f ? dh1[i] : 0.f;
        }
    }
    s_loss[threadIdx.x] = loss;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s_loss[threadIdx.x] += s_loss[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss_acc, s_loss[0]);
}

// One thread per parameter: sum of its per-sample gradient over the batch.
__global__ __launch_bounds__(256) void k_grad(const float* X, const int32_t* idx, int B, const float* H1,
                                              const float* H2, const float* DH1, const float* DH2, const float* DY,
                                              float* grad) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    float acc = 0.f;
    if (p < kOffB1) {
        const int i = p / kMlpIn, k = p % kMlpIn;
        for (int b = 0; b < B; ++b) acc = fmaf(DH1[(int64_t)b * kMlpH + i], X[(int64_t)idx[b] * kMlpIn + k], acc);
    } else if (p < kOffW2) {
        const int i = p - kOffB1;
        for (int b = 0; b < B; ++b) acc += DH1[(int64_t)b * kMlpH + i];
    } else if (p < kOffB2) {
        const int jj = (p - kOffW2) / kMlpH, i = (p - kOffW2) % kMlpH;
        for (int b = 0; b < B; ++b) acc = fmaf(DH2[(int64_t)b * kMlpH + jj], H1[(int64_t)b * kMlpH + i], acc);
    } else if (p < kOffW3) {
        const int jj = p - kOffB2;
        for (int b = 0; b < B; ++b) acc += DH2[(int64_t)b * kMlpH + jj];
    } else if (p < kOffB3) {
        const int jj = p - kOffW3;
        for (int b = 0; b < B; ++b) acc = fmaf(DY[b], H2[(int64_t)b * kMlpH + jj], acc);
    } else {
        for (int b = 0; b < B; ++b) acc += DY[b];
    }
    grad[p] = acc;
}

__global__ __launch_bounds__(256) void k_adamw(float* master, float* m, float* v, const float* grad, float lr,
                                               float beta1, float beta2, float eps, float wd, float bc1, float bc2,
                                               float* wbf, uint16_t* w16) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.f - beta1) * g;
    const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const bool is_weight = p < kOffB1 || (p >= kOffW2 && p < kOffB2) || (p >= kOffW3 && p < kOffB3);
    float x = master[p];
    x -= lr * ((mm / bc1) / (sqrtf(vv / bc2) + eps) + (is_weight ? wd * x : 0.f));
    master[p] = x;
    wbf[p] = bf16_round(x);
    if (w16 && frag_slot(p) >= 0) w16[frag_slot(p)] = bf16_bits(x);
}

__global__ __launch_bounds__(256) void k_round_params(const float* master, float* wbf, uint16_t* w16) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kMlpParams) {
        wbf[p] = bf16_round(master[p]);
        if (w16 && frag_slot(p) >= 0) w16[frag_slot(p)] = bf16_bits(master[p]);
    }
}

// ---------------------------------------------------------------------------
// near-queue binning (counting sort by depth bin)
// ---------------------------------------------------------------------------
__device__ inline uint64_t queue_len(const NearQueue& nq) {
    const unsigned long long n = *nq.count;
    return n < nq.cap ? n : nq.cap;
}

__global__ __launch_bounds__(256) void k_bin_count(Segs sg, Points pts, NearQueue nq, const uint8_t* seg_per,
                                                   double eps, int mode, const float* __restrict__ w,
                                                   const float* __restrict__ norm, const uint8_t* measured,
                                                   uint8_t* bins, uint32_t* wg_hist) {
    __shared__ uint32_t s_hist[kBins];
    if (threadIdx.x < kBins) s_hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t n = queue_len(nq);
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = (uint64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        int bin;
        if (mode == 2) {
            bin = measured[i];
        } else {
            uint32_t s;
            double qx, qy;
            queue_query(pts, nq, seg_per, i, s, qx, qy);
            float f[kMlpIn];
            pair_features(sg, s, qx, qy, eps, f);
            float d;
            if (mode == 1) {
                d = heuristic_depth(f, (float)eps);
            } else {
                float h1[kMlpH];
                standardise(f, norm);
                d = mlp_forward(w, f, h1);
            }
            bin = (int)rintf(d);
        }
        bin = bin < 0 ? 0 : (bin >= kBins ? kBins - 1 : bin);
        bins[i] = (uint8_t)bin;
        atomicAdd(&s_hist[bin], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kBins) wg_hist[(size_t)blockIdx.x * kBins + threadIdx.x] = s_hist[threadIdx.x];
}

// ---------------------------------------------------------------------------
// MLP inference on the matrix cores (v_mfma_f32_16x16x32_bf16: a 16 x 32 BF16
// tile times a 32 x 16 BF16 tile into a 16 x 16 FP32 tile).  Fragment layouts
// (lane l, element e):
//   A[i][k]  lane i + 16 (k / 8), element k % 8   (16 x 32)
//   B[k][j]  lane j + 16 (k / 8), element k % 8   (32 x 16)
//   C[i][j]  lane j + 16 (i / 4), element i % 4   (16 x 16)
// The network runs transposed, 16 rows (pairs) at a time: the weights are the
// A operands and the rows the N dimension, h1^T = W1 x^T (four 16-unit tiles,
// K = 16 inputs padded to 32) and h2^T = W2 h1^T (four tiles, two K steps).
// Lane (j, g) = j + 16 g then holds, for row j, hidden units 16 t + 4 g + e
// (e < 4) of every layer-1 tile t: eight of them per K step of layer 2.  As a
// contraction may take its K terms in any order, the layer-2 K step ks takes
// the lane's own units of tiles 2 ks and 2 ks + 1 (B element 4 (t % 2) + e)
// and W2's fragment columns are permuted alike, so the layer-1 accumulators
// (bias, ReLU, rounded to BF16) are layer 2's B operand without leaving the
// registers.  Layer 3 (one output) is a VALU dot product on the layer-2
// accumulators and a sum over the four lane groups.  Inputs, weights and
// layer-1 activations enter the matrix cores as BF16, accumulation in FP32.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct MlpFrags {
    bf16x8 a1[4];     // W1 tile t: lane (i, g) holds W1[16 t + i][8 g .. 8 g + 7] (zero for g >= 2)
    bf16x8 a2[4][2];  // W2 tile t, K step ks: lane (i, g) holds W2[16 t + i][l2_unit(ks, g, e)]
    f32x4 bias1[4], bias2[4], w3[4];  // element e of tile t: unit 16 t + 4 g + e
    float b3;
};

// w16: the fragment-order copy (frag_slot), 16-byte aligned.
__device__ inline void load_frags(const uint16_t* __restrict__ w16, const float* __restrict__ w, int lane,
                                  MlpFrags& F) {
    const int g = lane >> 4;
    const bf16x8* fr = reinterpret_cast<const bf16x8*>(w16);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        F.a1[t] = fr[t * 64 + lane];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) F.a2[t][ks] = fr[(4 + 2 * t + ks) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int u = 16 * t + 4 * g + e;
            F.bias1[t][e] = w[kOffB1 + u];
            F.bias2[t][e] = w[kOffB2 + u];
            F.w3[t][e] = w[kOffW3 + u];
        }
    }
    F.b3 = w[kOffB3];
}

// y of 16 rows: xb is lane (j, g)'s layer-1 B operand (row j's inputs
// 8 g .. 8 g + 7, zero for g >= 2).  Every lane of column j returns row j's y.
__device__ inline float mlp16(const MlpFrags& F, bf16x8 xb) {
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    bf16x8 hb[2];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a1[t], xb, zero, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) hb[t >> 1][4 * (t & 1) + e] = (__bf16)fmaxf(c[e] + F.bias1[t][e], 0.f);
    }
    float part = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2[t][0], hb[0], zero, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2[t][1], hb[1], c, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) part = fmaf(F.w3[t][e], fmaxf(c[e] + F.bias2[t][e], 0.f), part);
    }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    return part + F.b3;
}

// One wave, 64 rows: lane p's row (its 16 standardised features f) is row
// p % 16 of block p / 16; the features cross lanes through sx (64 rows of
// 16 BF16, this wave's own LDS; LDS operations of a wave complete in order).
__device__ inline float mlp_wave(const MlpFrags& F, const float* f, bf16x8* sx, int lane) {
    bf16x8 lo, hi;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        lo[k] = (__bf16)f[k];
        hi[k] = (__bf16)f[8 + k];
    }
    sx[2 * lane] = lo;
    sx[2 * lane + 1] = hi;
    __builtin_amdgcn_wave_barrier();
    const int j = lane & 15, g = lane >> 4;
    float mine = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        bf16x8 xb = sx[2 * (16 * b + j) + (g & 1)];
        if (g >= 2) xb = bf16x8{};
        const float y = mlp16(F, xb);
        if (g == b) mine = y;
    }
    __builtin_amdgcn_wave_barrier();
    return mine;
}

// Bin counts of the near queue with the MLP on the matrix cores: a wave
// forms the standardised features of 64 entries (one per lane), runs
// mlp_wave and bins the predictions like k_bin_count.
__global__ __launch_bounds__(256) void k_bin_count_mfma(Segs sg, Points pts, NearQueue nq, const uint8_t* seg_per,
                                                        double eps, const uint16_t* __restrict__ w16,
                                                        const float* __restrict__ w, const float* __restrict__ norm,
                                                        uint8_t* bins, uint32_t* wg_hist) {
    __shared__ uint32_t s_hist[kBins];
    __shared__ bf16x8 s_x[4][2 * kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < kBins) s_hist[threadIdx.x] = 0;
    __syncthreads();
    MlpFrags F;
    load_frags(w16, w, lane, F);
    const uint64_t n = queue_len(nq);
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = (uint64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    for (uint64_t base = b0 + (uint64_t)wave * kWave; base < b1; base += 4 * kWave) {
        const uint64_t i = base + lane;
        const bool ok = i < b1;
        float f[kMlpIn];
        if (ok) {
            uint32_t s;
            double qx, qy;
            queue_query(pts, nq, seg_per, i, s, qx, qy);
            pair_features(sg, s, qx, qy, eps, f);
            standardise(f, norm);
        } else {
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k) f[k] = 0.f;
        }
        const float y = mlp_wave(F, f, s_x[wave], lane);
        if (ok) {
            int bin = (int)rintf(y);
            bin = bin < 0 ? 0 : (bin >= kBins ? kBins - 1 : bin);
            bins[i] = (uint8_t)bin;
            atomicAdd(&s_hist[bin], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kBins) wg_hist[(size_t)blockIdx.x * kBins + threadIdx.x] = s_hist[threadIdx.x];
}

// Predictions of standardised features X [n][16] on the matrix cores:
// persistent waves, 64 rows per wave and step.
__global__ __launch_bounds__(256) void k_predict_mfma(const uint16_t* __restrict__ w16, const float* __restrict__ w,
                                                      const float* __restrict__ X, int64_t n, float* out) {
    __shared__ bf16x8 s_x[4][2 * kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    MlpFrags F;
    load_frags(w16, w, lane, F);
    const int64_t tiles = (n + kWave - 1) / kWave;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t i = tile * kWave + lane;
        float f[kMlpIn];
        if (i < n) {
            const float4* x = reinterpret_cast<const float4*>(X + i * kMlpIn);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float4 v = x[k];
                f[4 * k] = v.x;
                f[4 * k + 1] = v.y;
                f[4 * k + 2] = v.z;
                f[4 * k + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k) f[k] = 0.f;
        }
        const float y = mlp_wave(F, f, s_x[wave], lane);
        if (i < n) out[i] = y;
    }
}

// wg_hist[g][b] -> start offset of (g, b) in bin-major order (in place).
// One workgroup, thread g owns workgroup g's counts (G <= 1024); per bin a
// block-wide exclusive scan over g.
__global__ __launch_bounds__(1024) void k_bin_scan(uint32_t* wg_hist, int G) {
    __shared__ uint32_t s_v[1024];
    __shared__ uint32_t s_base;
    const int g = threadIdx.x;
    if (g == 0) s_base = 0;
    for (int b = 0; b < kBins; ++b) {
        const uint32_t c = g < G ? wg_hist[(size_t)g * kBins + b] : 0u;
        s_v[g] = c;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t t = g >= off ? s_v[g - off] : 0u;
            __syncthreads();
            s_v[g] += t;
            __syncthreads();
        }
        const uint32_t incl = s_v[g];
        const uint32_t base = s_base;
        if (g < G) wg_hist[(size_t)g * kBins + b] = base + incl - c;
        __syncthreads();
        if (g == 1023) s_base = base + incl;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_bin_scatter(NearQueue nq, const uint8_t* bins, const uint32_t* wg_off,
                                                     uint2* qs_out, double2* sh_out) {
    __shared__ uint32_t s_cur[kBins];
    if (threadIdx.x < kBins) s_cur[threadIdx.x] = wg_off[(size_t)blockIdx.x * kBins + threadIdx.x];
    __syncthreads();
    const uint64_t n = queue_len(nq);
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = (uint64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        const uint32_t pos = atomicAdd(&s_cur[bins[i]], 1u);
        if (pos < nq.cap) {
            qs_out[pos] = nq.qs[i];
            if (nq.shift) sh_out[pos] = nq.shift[i];
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_pair_features(const Segs& sg, const Points& pts, const int32_t* pp, const int32_t* ps, int64_t n,
                                double eps, float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sg, pts, pp, ps, n, eps,
                       out);
    return hipGetLastError();
}

hipError_t launch_queue_features(const Segs& sg, const Points& pts, NearQueue nq, const uint8_t* seg_per, double eps,
                                 uint64_t limit, float* out, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_queue_features, dim3(grid), dim3(256), 0, st, sg, pts, nq, seg_per, eps, limit, out);
    return hipGetLastError();
}

hipError_t launch_predict(const float* w, const float* X, int64_t n, float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, X, n, out);
    return hipGetLastError();
}

hipError_t launch_train_step(const float* w, const float* X, const float* Y, const int32_t* idx, int B, float delta,
                             TrainBufs tb, hipStream_t st) {
    hipLaunchKernelGGL(k_fwd_bwd, dim3((B + 255) / 256), dim3(256), 0, st, w, X, Y, idx, B, delta, tb.H1, tb.H2,
                       tb.DH1, tb.DH2, tb.DY, tb.loss);
    hipLaunchKernelGGL(k_grad, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, X, idx, B, tb.H1, tb.H2, tb.DH1,
                       tb.DH2, tb.DY, tb.grad);
    return hipGetLastError();
}

hipError_t launch_adamw(float* master, float* m, float* v, const float* grad, float lr, float beta1, float beta2,
                        float eps, float wd, int step, float* wbf, uint16_t* w16, hipStream_t st) {
    const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adamw, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, master, m, v, grad, lr, beta1,
                       beta2, eps, wd, bc1, bc2, wbf, w16);
    return hipGetLastError();
}

hipError_t launch_predict_mfma(const uint16_t* w16, const float* w, const float* X, int64_t n, float* out, int cus,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    // persistent: at most eight workgroups per compute unit
    const int64_t want = (n + 4 * kWave - 1) / (4 * kWave);
    const unsigned grid = (unsigned)(want < 8 * (int64_t)cus ? want : 8 * (int64_t)cus);
    hipLaunchKernelGGL(k_predict_mfma, dim3(grid), dim3(256), 0, st, w16, w, X, n, out);
    return hipGetLastError();
}

hipError_t launch_round_params(const float* master, float* wbf, uint16_t* w16, hipStream_t st) {
    hipLaunchKernelGGL(k_round_params, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, master, wbf, w16);
    return hipGetLastError();
}

hipError_t launch_binning(const Segs& sg, const Points& pts, NearQueue nq, const uint8_t* seg_per, double eps,
                          int mode, const float* w, const uint16_t* w16, const float* norm, const uint8_t* measured,
                          uint8_t* bins, uint32_t* wg_hist, int G, uint2* qs_out, double2* sh_out, hipStream_t st) {
    if (mode == 0 && w16)  // the MLP on the matrix cores
        hipLaunchKernelGGL(k_bin_count_mfma, dim3(G), dim3(256), 0, st, sg, pts, nq, seg_per, eps, w16, w, norm, bins,
                           wg_hist);
    else
        hipLaunchKernelGGL(k_bin_count, dim3(G), dim3(256), 0, st, sg, pts, nq, seg_per, eps, mode, w, norm,
                           measured, bins, wg_hist);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, wg_hist, G);
    hipLaunchKernelGGL(k_bin_scatter, dim3(G), dim3(256), 0, st, nq, bins, wg_hist, qs_out, sh_out);
    return hipGetLastError();
}

}  // namespace wn
