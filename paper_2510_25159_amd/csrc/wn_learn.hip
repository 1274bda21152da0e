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
                                               float* wbf) {
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
}

__global__ __launch_bounds__(256) void k_round_params(const float* master, float* wbf) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kMlpParams) wbf[p] = bf16_round(master[p]);
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
                        float eps, float wd, int step, float* wbf, hipStream_t st) {
    const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adamw, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, master, m, v, grad, lr, beta1,
                       beta2, eps, wd, bc1, bc2, wbf);
    return hipGetLastError();
}

hipError_t launch_round_params(const float* master, float* wbf, hipStream_t st) {
    hipLaunchKernelGGL(k_round_params, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, master, wbf);
    return hipGetLastError();
}

hipError_t launch_binning(const Segs& sg, const Points& pts, NearQueue nq, const uint8_t* seg_per, double eps,
                          int mode, const float* w, const float* norm, const uint8_t* measured, uint8_t* bins,
                          uint32_t* wg_hist, int G, uint2* qs_out, double2* sh_out, hipStream_t st) {
    hipLaunchKernelGGL(k_bin_count, dim3(G), dim3(256), 0, st, sg, pts, nq, seg_per, eps, mode, w, norm, measured,
                       bins, wg_hist);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, wg_hist, G);
    hipLaunchKernelGGL(k_bin_scatter, dim3(G), dim3(256), 0, st, nq, bins, wg_hist, qs_out, sh_out);
    return hipGetLastError();
}

}  // namespace wn
