// Host API of the learned depth predictor: creation, parameters, the GPU
// training driver (labels = depths the near pass itself records), loss and
// gradient for checks, prediction, pair features.
#include "wn_host_internal.h"
#include "wn_learn.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <vector>

using namespace wn;

namespace {

hipError_t upload_params(wn_predictor* p, const float* params, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(p->d_master, params, kMlpParams * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_round_params(p->d_master, p->d_wbf, p->d_w16, st);
    return e;
}

float mean_abs(const std::vector<float>& a, const std::vector<float>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += fabs((double)a[i] - (double)b[i]);
    return a.empty() ? 0.f : (float)(s / (double)a.size());
}

}  // namespace

extern "C" {

wn_status wn_predictor_create(int32_t seed, wn_predictor** out) {
    if (!out) return WN_E_INVALID;
    *out = nullptr;
    wn_predictor* p = new (std::nothrow) wn_predictor();
    if (!p) return WN_E_NOMEM;
    const size_t bytes = (size_t)kMlpFragSlots * 2 + (size_t)kMlpParams * 4 * 4 + 2 * kMlpIn * 4 + 1024;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess) e = hipMalloc(&p->dmem, bytes);
    if (e != hipSuccess) {
        delete p;
        return hip_status(e);
    }
    char* b = (char*)p->dmem;
    p->d_w16 = reinterpret_cast<uint16_t*>(b);  // first: 16-byte fragment loads
    p->d_master = reinterpret_cast<float*>(b + (size_t)kMlpFragSlots * 2);
    p->d_m = p->d_master + kMlpParams;
    p->d_v = p->d_m + kMlpParams;
    p->d_wbf = p->d_v + kMlpParams;
    p->d_norm = p->d_wbf + kMlpParams;
    // He-uniform initialisation of the weights, zero biases (host, seeded)
    std::vector<float> prm((size_t)kMlpParams, 0.f);
    std::mt19937_64 rng((uint64_t)seed * 0x9E3779B97F4A7C15ull + 12345u);
    auto fill = [&](int off, int count, int fan_in) {
        const double a = sqrt(6.0 / fan_in);
        std::uniform_real_distribution<double> U(-a, a);
        for (int i = 0; i < count; ++i) prm[off + i] = (float)U(rng);
    };
    fill(kOffW1, kMlpH * kMlpIn, kMlpIn);
    fill(kOffW2, kMlpH * kMlpH, kMlpH);
    fill(kOffW3, kMlpH, kMlpH);
    std::vector<float> norm(2 * kMlpIn, 0.f);
    for (int k = 0; k < kMlpIn; ++k) norm[kMlpIn + k] = 1.f;
    e = hipMemset(p->d_m, 0, kMlpParams * 4 * 2);
    // the fragment slots no weight maps to (layer 1's K padding) stay zero
    if (e == hipSuccess) e = hipMemset(p->d_w16, 0, (size_t)kMlpFragSlots * 2);
    if (e == hipSuccess) e = hipMemcpy(p->d_norm, norm.data(), norm.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = upload_params(p, prm.data(), nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        wn_predictor_destroy(p);
        return hip_status(e);
    }
    *out = p;
    return WN_OK;
}

void wn_predictor_destroy(wn_predictor* p) {
    if (!p) return;
    if (p->dmem) (void)hipFree(p->dmem);
    delete p;
}

wn_status wn_predictor_get_params(const wn_predictor* p, float* params, float* norm) {
    if (!p) return WN_E_INVALID;
    hipError_t e = hipSuccess;
    if (params) e = hipMemcpy(params, p->d_master, kMlpParams * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && norm) e = hipMemcpy(norm, p->d_norm, 2 * kMlpIn * 4, hipMemcpyDeviceToHost);
    return hip_status(e);
}

wn_status wn_predictor_set_params(wn_predictor* p, const float* params, const float* norm) {
    if (!p) return WN_E_INVALID;
    if (norm)
        for (int k = 0; k < kMlpIn; ++k)
            if (!(norm[kMlpIn + k] > 0.f) || !isfinite(norm[k])) return WN_E_INVALID;
    if (params)
        for (int i = 0; i < kMlpParams; ++i)
            if (!isfinite(params[i])) return WN_E_INVALID;
    hipError_t e = hipSuccess;
    if (params) e = upload_params(p, params, nullptr);
    if (e == hipSuccess && norm) e = hipMemcpy(p->d_norm, norm, 2 * kMlpIn * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return hip_status(e);
}

wn_status wn_predictor_predict(const wn_predictor* p, const float* X, int64_t n, float* out, void* stream) {
    if (!p || n < 0 || (n > 0 && (!X || !out))) return WN_E_INVALID;
    return hip_status(launch_predict(p->d_wbf, X, n, out, (hipStream_t)stream));
}

wn_status wn_predictor_predict_mfma(const wn_predictor* p, const float* X, int64_t n, float* out, void* stream) {
    if (!p || n < 0 || (n > 0 && (!X || !out)) || (reinterpret_cast<uintptr_t>(X) & 15)) return WN_E_INVALID;
    return hip_status(launch_predict_mfma(p->d_w16, p->d_wbf, X, n, out, p->cu_count, (hipStream_t)stream));
}

wn_status wn_predictor_loss_grad(const wn_predictor* p, const float* X, const float* Y, int64_t n, float delta,
                                 float* loss, float* grad, void* stream) {
    if (!p || !X || !Y || n < 1 || n > (1 << 24) || !(delta > 0.f)) return WN_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const int B = (int)n;
    const size_t act = (size_t)B * kMlpH * 4;
    void* buf = nullptr;
    hipError_t e = hipMalloc(&buf, 4 * act + (size_t)B * 4 + kMlpParams * 4 + 256 + (size_t)B * 4);
    if (e != hipSuccess) return hip_status(e);
    char* b = (char*)buf;
    TrainBufs tb{(float*)b, (float*)(b + act), (float*)(b + 2 * act), (float*)(b + 3 * act), (float*)(b + 4 * act),
                 (float*)(b + 4 * act + (size_t)B * 4), (float*)(b + 4 * act + (size_t)B * 4 + kMlpParams * 4)};
    int32_t* idx = (int32_t*)(b + 4 * act + (size_t)B * 4 + kMlpParams * 4 + 256);
    std::vector<int32_t> hidx((size_t)B);
    for (int i = 0; i < B; ++i) hidx[i] = i;
    e = hipMemcpyAsync(idx, hidx.data(), (size_t)B * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(tb.loss, 0, 4, st);
    if (e == hipSuccess) e = launch_train_step(p->d_wbf, X, Y, idx, B, delta, tb, st);
    float l = 0.f;
    if (e == hipSuccess) e = hipMemcpyAsync(&l, tb.loss, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && grad) e = hipMemcpyAsync(grad, tb.grad, kMlpParams * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e == hipSuccess && loss) *loss = l / (float)B;
    return hip_status(e);
}

wn_status wn_pair_features(const wn_faces* h, const wn_points* pts, const int32_t* pp, const int32_t* ps, int64_t n,
                           float* out, void* stream) {
    if (!h || !pts || n < 0 || (n > 0 && (!pp || !ps || !out || !pts->u || !pts->v))) return WN_E_INVALID;
    const Points P{pts->u, pts->v, pts->stride, pts->face_point_offsets, pts->num_points};
    return hip_status(launch_pair_features(h->sg, P, pp, ps, n, h->eps, out, (hipStream_t)stream));
}

wn_status wn_near_pairs(const wn_faces* h, const wn_points* p, int64_t capacity, int32_t* pair_point,
                        int32_t* pair_segment, uint8_t* pair_depth, double* pair_shift, int64_t* out_count,
                        int32_t bound, void* stream) {
    if (!h || !p || !out_count || capacity < 0) return WN_E_INVALID;
    if (bound != WN_BOUND_GLOBAL && bound != WN_BOUND_SUBDIVIDED) return WN_E_INVALID;
    if (capacity > 0 && (!pair_point || !pair_segment || !pair_depth)) return WN_E_INVALID;
    const int64_t N = p->num_points;
    if (N < 0 || N >= 0x7fffffffll) return WN_E_INVALID;
    *out_count = 0;
    if (N == 0) return WN_OK;
    if (!p->u || !p->v || p->stride < 1 || !p->face_point_offsets) return WN_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const Points pts{p->u, p->v, p->stride, p->face_point_offsets, N};
    // a queue that holds every near pair of these points (a pair that does not
    // fit would be recomputed in line and never logged)
    const int64_t cap = std::min<int64_t>(std::max<int64_t>(8 * N + 65536, capacity), (int64_t)1 << 34);
    Scratch sc;
    hipError_t e = scratch_alloc(h, N, cap, false, false, nullptr, nullptr, h->rule, sc, st, true);
    if (e != hipSuccess) return hip_status(e);
    uint8_t* d_depth = nullptr;
    e = hipMallocAsync((void**)&d_depth, (size_t)cap, st);
    if (e == hipSuccess) e = far_passes(h, pts, 256, 1, false, 0, sc, nullptr, st);
    if (e == hipSuccess) e = near_pass(h, pts, sc.nq, sc.out, nullptr, d_depth, nullptr, st, near_cursor(sc, 0),
                                                  bound == WN_BOUND_SUBDIVIDED);
    unsigned long long cnt = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, sc.nq.count, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const bool overflow = cnt > (unsigned long long)cap;
    const int64_t n = std::min<int64_t>((int64_t)std::min<unsigned long long>(cnt, (unsigned long long)cap), capacity);
    if (e == hipSuccess && n > 0) {
        e = launch_split_pairs(sc.nq.qs, n, pair_point, pair_segment, st);
        if (e == hipSuccess) e = hipMemcpyAsync(pair_depth, d_depth, (size_t)n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && pair_shift) {
            if (sc.nq.shift)
                e = hipMemcpyAsync(pair_shift, sc.nq.shift, (size_t)n * 16, hipMemcpyDeviceToDevice, st);
            else
                e = hipMemsetAsync(pair_shift, 0, (size_t)n * 16, st);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFreeAsync(d_depth, st);
    scratch_free(sc, st);
    if (e != hipSuccess) return hip_status(e);
    if (overflow) return WN_E_NOMEM;
    *out_count = (int64_t)cnt;
    return WN_OK;
}

wn_status wn_predictor_train(wn_predictor* pr, const wn_faces* h, const wn_points* p, const wn_train_opts* opts_in,
                             wn_train_report* report, void* stream) {
    if (!pr || !h || !p) return WN_E_INVALID;
    wn_train_opts o{};
    if (opts_in) o = *opts_in;
    if (o.epochs <= 0) o.epochs = 8;
    if (o.batch <= 0) o.batch = 4096;
    if (!(o.lr > 0.f)) o.lr = 2e-3f;
    if (!(o.weight_decay >= 0.f)) o.weight_decay = 1e-4f;
    if (o.weight_decay == 0.f && !opts_in) o.weight_decay = 1e-4f;
    if (!(o.huber_delta > 0.f)) o.huber_delta = 1.f;
    if (!(o.holdout > 0.f && o.holdout < 0.9f)) o.holdout = 0.1f;
    if (o.batch > (1 << 20) || o.epochs > 10000) return WN_E_INVALID;
    const int64_t N = p->num_points;
    const int32_t F = h->num_faces;
    if (N <= 0 || N >= 0x7fffffffll || !p->u || !p->v || p->stride < 1 || !p->face_point_offsets) return WN_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const Points pts{p->u, p->v, p->stride, p->face_point_offsets, N};
    const int64_t cap = std::min<int64_t>(8 * N + 65536, (int64_t)1 << 34);

    // 1. near pairs of the training points and their measured depths
    Scratch sc;
    hipError_t e = scratch_alloc(h, N, cap, false, false, nullptr, nullptr, h->rule, sc, st, true);
    if (e != hipSuccess) return hip_status(e);
    uint8_t* d_depth = nullptr;
    e = hipMallocAsync((void**)&d_depth, (size_t)cap, st);
    if (e == hipSuccess) e = far_passes(h, pts, 256, 1, false, 0, sc, nullptr, st);
    if (e == hipSuccess) e = near_pass(h, pts, sc.nq, sc.out, nullptr, d_depth, nullptr, st, near_cursor(sc, 0));
    unsigned long long cnt = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, sc.nq.count, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int64_t n = (int64_t)std::min<unsigned long long>(cnt, (unsigned long long)cap);
    if (o.max_samples > 0) n = std::min<int64_t>(n, o.max_samples);
    n = std::min<int64_t>(n, (int64_t)1 << 26);
    float* d_feat = nullptr;
    if (e == hipSuccess && n > 0) e = hipMallocAsync((void**)&d_feat, (size_t)n * kMlpIn * 4, st);
    if (e == hipSuccess && n > 0)
        e = launch_queue_features(h->sg, pts, sc.nq, h->pt.seg_periodic, h->eps, (uint64_t)n, d_feat,
                                  h->cu_count * 4, st);
    std::vector<float> feat((size_t)n * kMlpIn);
    std::vector<uint8_t> dep((size_t)n);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(feat.data(), d_feat, feat.size() * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(dep.data(), d_depth, (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (d_feat) (void)hipFreeAsync(d_feat, st);
    if (d_depth) (void)hipFreeAsync(d_depth, st);
    scratch_free(sc, st);
    if (e != hipSuccess) return hip_status(e);
    if (n < 16) return WN_E_INVALID;  // nothing to learn from

    // 2. standardisation, seeded split
    std::vector<double> mu(kMlpIn, 0.0), sd(kMlpIn, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < kMlpIn; ++k) mu[k] += feat[(size_t)i * kMlpIn + k];
    for (int k = 0; k < kMlpIn; ++k) mu[k] /= (double)n;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < kMlpIn; ++k) {
            const double d = feat[(size_t)i * kMlpIn + k] - mu[k];
            sd[k] += d * d;
        }
    std::vector<float> norm(2 * kMlpIn);
    for (int k = 0; k < kMlpIn; ++k) {
        norm[k] = (float)mu[k];
        norm[kMlpIn + k] = (float)std::max(sqrt(sd[k] / (double)n), 1e-6);
    }
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    std::mt19937_64 rng((uint64_t)o.seed * 0x2545F4914F6CDD1Dull + 7u);
    std::shuffle(perm.begin(), perm.end(), rng);
    const int64_t n_hold = std::max<int64_t>(1, (int64_t)(o.holdout * (double)n));
    const int64_t n_train = n - n_hold;
    std::vector<float> Xs((size_t)n * kMlpIn), Y((size_t)n);
    double ymean = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = perm[r];
        for (int k = 0; k < kMlpIn; ++k)
            Xs[(size_t)r * kMlpIn + k] = (feat[(size_t)i * kMlpIn + k] - norm[k]) / norm[kMlpIn + k];
        Y[r] = (float)dep[i];
        if (r < n_train) ymean += Y[r];
    }
    ymean /= (double)std::max<int64_t>(n_train, 1);

    // 3. training on the GPU
    const int B = (int)std::min<int64_t>(o.batch, n_train);
    const size_t act = (size_t)B * kMlpH * 4;
    void* buf = nullptr;
    const size_t bytes = (size_t)n * kMlpIn * 4 + (size_t)n * 4 + (size_t)n * 4 + 4 * act + (size_t)B * 4 +
                         kMlpParams * 4 + 1024;
    e = hipMalloc(&buf, bytes);
    if (e != hipSuccess) return hip_status(e);
    char* b = (char*)buf;
    float* dX = (float*)b;
    float* dY = (float*)(b + (size_t)n * kMlpIn * 4);
    int32_t* dIdx = (int32_t*)(b + (size_t)n * kMlpIn * 4 + (size_t)n * 4);
    char* t0 = b + (size_t)n * kMlpIn * 4 + (size_t)n * 8;
    TrainBufs tb{(float*)t0, (float*)(t0 + act), (float*)(t0 + 2 * act), (float*)(t0 + 3 * act),
                 (float*)(t0 + 4 * act), (float*)(t0 + 4 * act + (size_t)B * 4),
                 (float*)(t0 + 4 * act + (size_t)B * 4 + kMlpParams * 4)};
    e = hipMemcpyAsync(dX, Xs.data(), Xs.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dY, Y.data(), Y.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pr->d_norm, norm.data(), norm.size() * 4, hipMemcpyHostToDevice, st);
    // start the output bias at the mean depth
    std::vector<float> prm((size_t)kMlpParams);
    if (e == hipSuccess) e = hipMemcpyAsync(prm.data(), pr->d_master, kMlpParams * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        prm[kOffB3] = (float)ymean;
        e = upload_params(pr, prm.data(), st);
    }
    if (e == hipSuccess) e = hipMemsetAsync(pr->d_m, 0, kMlpParams * 4 * 2, st);
    pr->step = 0;
    std::vector<int32_t> ep((size_t)n_train);
    float last_loss = 0.f;
    int steps = 0;
    for (int epoch = 0; epoch < o.epochs && e == hipSuccess; ++epoch) {
        for (int64_t i = 0; i < n_train; ++i) ep[i] = (int32_t)i;
        std::shuffle(ep.begin(), ep.end(), rng);
        e = hipMemcpyAsync(dIdx, ep.data(), (size_t)n_train * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(tb.loss, 0, 4, st);
        int nb = 0;
        for (int64_t s0 = 0; s0 + B <= n_train && e == hipSuccess; s0 += B, ++nb) {
            e = launch_train_step(pr->d_wbf, dX, dY, dIdx + s0, B, o.huber_delta, tb, st);
            if (e == hipSuccess)
                e = launch_adamw(pr->d_master, pr->d_m, pr->d_v, tb.grad, o.lr, 0.9f, 0.999f, 1e-8f, o.weight_decay,
                                 ++pr->step, pr->d_wbf, pr->d_w16, st);
            ++steps;
        }
        float l = 0.f;
        if (e == hipSuccess) e = hipMemcpyAsync(&l, tb.loss, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        last_loss = nb > 0 ? l / (float)(nb * B) : 0.f;
    }
    // 4. holdout report
    std::vector<float> pred((size_t)n_hold), yh((size_t)n_hold), base((size_t)n_hold, (float)ymean), heur((size_t)n_hold);
    float* dP = tb.DY;  // reuse: B >= 1 floats... holdout may be larger: allocate
    float* dPh = nullptr;
    if (e == hipSuccess) e = hipMalloc(&dPh, (size_t)n_hold * 4);
    if (e == hipSuccess) e = launch_predict(pr->d_wbf, dX + (size_t)n_train * kMlpIn, n_hold, dPh, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pred.data(), dPh, (size_t)n_hold * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)dP;
    if (dPh) (void)hipFree(dPh);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_status(e);
    for (int64_t r = 0; r < n_hold; ++r) {
        yh[r] = Y[n_train + r];
        const int64_t i = perm[n_train + r];
        heur[r] = heuristic_depth(&feat[(size_t)i * kMlpIn], (float)h->eps);
    }
    if (report) {
        report->samples = n;
        report->train_samples = n_train;
        report->steps = steps;
        report->final_train_loss = last_loss;
        report->holdout_mae = mean_abs(pred, yh);
        report->baseline_mae = mean_abs(base, yh);
        report->heuristic_mae = mean_abs(heur, yh);
        report->mean_depth = (float)ymean;
    }
    return WN_OK;
}

}  // extern "C"
