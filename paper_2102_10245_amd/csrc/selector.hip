// Execution choice for an MTTKRP: the learned selector (a perceptron with
// two hidden ReLU layers that predicts log2 run time for every candidate
// (strategy, L)) when weights are installed and the tensor lies inside the
// feature range it was trained on; otherwise the fiber-reuse rule of
// Section 3.3 (local staging when nnz / I_n > 4, atomics otherwise).
// Inference here is on the host: one query is ~6K multiply-adds, far
// cheaper than a kernel launch and a device-to-host copy; the HIP kernels
// in mlp.hip run the same network in batch for training and evaluation.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "common.h"

namespace alto {
namespace {

constexpr int kF = 15;

struct Selector {
    bool loaded = false;
    int F = 0, H = 0, K = 0, nL = 0;
    std::vector<float> mean, scale, fmin, fmax, Ls, W1, b1, W2, b2, W3, b3;
};

std::mutex g_sel_mu;
Selector g_sel;

void features(const alto_tensor *t, int mode, int R, int prec, float *f) {
    const double I = (double)t->dims[mode];
    const double M = (double)std::max<int64_t>(1, t->nnz);
    double sum_other = 0.0, max_other = 1.0, min_other = 1e300;
    for (int m = 0; m < t->N; m++) {
        if (m == mode) continue;
        sum_other += (double)t->dims[m];
        max_other = std::max(max_other, (double)t->dims[m]);
        min_other = std::min(min_other, (double)t->dims[m]);
    }
    const double fbytes = prec == ALTO_PREC_BF16 ? 2.0 : 4.0;
    f[0] = (float)std::log2(I);
    f[1] = (float)std::log2(M);
    f[2] = (float)std::log2(M / I);
    f[3] = (float)t->N;
    f[4] = (float)std::log2((double)R);
    f[5] = (float)prec;
    f[6] = (float)t->B / 32.f;
    f[7] = (float)t->key_bits / 64.f;
    f[8] = (float)std::log2(std::max(1.0, sum_other));
    f[9] = (float)std::log2(max_other);
    f[10] = (float)std::log2(min_other * R * fbytes);  // smallest gathered factor matrix, bytes
    f[11] = (float)std::log2(I * R);
    f[12] = t->row_hot[mode];       // skew of the output mode
    f[13] = t->row_distinct[mode];
    // The MTTKRP gathers the smallest other factor matrix from LDS when it
    // takes at most 64 KB and segments hold at least 65 536 nonzeros (see
    // fill_mt_launch): log2 of the largest segment count that still does, or
    // -1 when the matrix does not fit.
    const bool spec = R == 8 || R == 16 || R == 32 || R == 64;
    f[14] = spec && min_other * R * fbytes <= 65536.0 ? (float)std::log2(std::max(1.0, M / 65536.0)) : -1.f;
}

const int kOrder[3] = {ALTO_STRATEGY_ATOMIC, ALTO_STRATEGY_STAGED, ALTO_STRATEGY_SORTED};

void heuristic(const alto_tensor *t, int mode, alto_exec *out) {
    const double reuse = (double)t->nnz / (double)t->dims[mode];
    out->strategy = reuse > 4.0 ? ALTO_STRATEGY_STAGED : ALTO_STRATEGY_ATOMIC;
    out->num_segments = 0;
}

// candidates timed at most when the network's predictions are close
constexpr int kCloseMax = 3;

// margin of predicted log2 time under which the network's runners-up are
// timed too (ALTO_SELECT_MARGIN; 0, the default, trusts the argmin)
float close_margin() {
    const char *e = getenv("ALTO_SELECT_MARGIN");
    const float m = e && *e ? (float)atof(e) : 0.f;
    return m > 0.f ? m : 0.f;
}

// The plan of (tensor, mode, R, prec) and where it came from.
int select_impl(const alto_tensor *t, int mode, int R, int prec, alto_exec *out,
                std::vector<alto_exec> *close = nullptr) {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    if (!g_sel.loaded || t->nnz == 0) {
        heuristic(t, mode, out);
        return kPlanRule;
    }
    const Selector &s = g_sel;
    float f[kF];
    features(t, mode, R, prec, f);
    for (int q = 0; q < kF; q++) {
        const float span = s.fmax[q] - s.fmin[q];
        const float tol = 0.25f * span + 0.5f;
        if (f[q] < s.fmin[q] - tol || f[q] > s.fmax[q] + tol) {
            heuristic(t, mode, out);
            return kPlanOutside;
        }
    }
    std::vector<float> h1(s.H), h2(s.H);
    for (int j = 0; j < s.H; j++) {
        float a = s.b1[j];
        for (int q = 0; q < s.F; q++) a += s.W1[(size_t)j * s.F + q] * ((f[q] - s.mean[q]) / s.scale[q]);
        h1[j] = a > 0.f ? a : 0.f;
    }
    for (int j = 0; j < s.H; j++) {
        float a = s.b2[j];
        for (int q = 0; q < s.H; q++) a += s.W2[(size_t)j * s.H + q] * h1[q];
        h2[j] = a > 0.f ? a : 0.f;
    }
    std::vector<float> y(s.K);
    int best = 0;
    for (int k = 0; k < s.K; k++) {
        float a = s.b3[k];
        for (int q = 0; q < s.H; q++) a += s.W3[(size_t)k * s.H + q] * h2[q];
        y[k] = a;
        if (a < y[best]) best = k;
    }
    auto plan = [&](int k) { return alto_exec{kOrder[k / s.nL], (int)s.Ls[k % s.nL]}; };
    *out = plan(best);
    const float margin = close_margin();
    if (margin > 0.f) {
        // candidates predicted within the margin of the best, best first
        std::vector<int> ks;
        for (int k = 0; k < s.K; k++)
            if (y[k] <= y[best] + margin) ks.push_back(k);
        std::stable_sort(ks.begin(), ks.end(), [&](int a, int b) { return y[a] < y[b]; });
        if (ks.size() > (size_t)kCloseMax) ks.resize(kCloseMax);
        if (ks.size() > 1) {
            if (close) {
                close->clear();
                for (int k : ks) close->push_back(plan(k));
            }
            return kPlanClose;
        }
    }
    return kPlanNet;
}

}  // namespace

int select_plan(const alto_tensor *t, int mode, int R, int prec, alto_exec *out, std::vector<alto_exec> *close) {
    return select_impl(t, mode, R, prec, out, close);
}

std::vector<alto_exec> selector_candidates() {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    std::vector<alto_exec> c;
    const int nL = g_sel.loaded ? g_sel.nL : 7;
    const int S = g_sel.loaded ? g_sel.K / g_sel.nL : 3;
    static const int kDefaultLs[7] = {256, 512, 1024, 2048, 4096, 8192, 16384};
    for (int st = 0; st < S; st++)
        for (int q = 0; q < nL; q++)
            c.push_back(alto_exec{kOrder[st], g_sel.loaded ? (int)g_sel.Ls[q] : kDefaultLs[q]});
    return c;
}

}  // namespace alto

using namespace alto;

extern "C" {

int alto_selector_features(const alto_tensor *t, int mode, int R, int prec, float *out) {
    if (!t || !out) return set_error(ALTO_E_INVAL, "null argument");
    if (mode < 0 || mode >= t->N) return set_error(ALTO_E_INVAL, "mode out of range");
    if (R < 1 || R > ALTO_MAX_RANK) return set_error(ALTO_E_INVAL, "R must be in 1..256");
    features(t, mode, R, prec, out);
    return ALTO_OK;
}

int alto_selector_load(const float *w, size_t n) {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    if (n == 0) {
        g_sel = Selector();
        return ALTO_OK;
    }
    if (!w || n < 4) return set_error(ALTO_E_INVAL, "selector weights too short");
    Selector s;
    s.F = (int)w[0];
    s.H = (int)w[1];
    s.K = (int)w[2];
    s.nL = (int)w[3];
    if (s.F != kF || s.H < 1 || s.H > 256 || s.nL < 1 || (s.K != 2 * s.nL && s.K != 3 * s.nL))
        return set_error(ALTO_E_INVAL, "selector header must be {15, H<=256, 2*nL or 3*nL, nL}");
    const size_t need = 4 + 4 * (size_t)s.F + s.nL + (size_t)s.H * s.F + s.H + (size_t)s.H * s.H + s.H +
                        (size_t)s.K * s.H + s.K;
    if (n != need) return set_error(ALTO_E_INVAL, "selector weight count does not match its header");
    const float *p = w + 4;
    auto take = [&](std::vector<float> &v, size_t c) {
        v.assign(p, p + c);
        p += c;
    };
    take(s.mean, s.F);
    take(s.scale, s.F);
    take(s.fmin, s.F);
    take(s.fmax, s.F);
    take(s.Ls, s.nL);
    take(s.W1, (size_t)s.H * s.F);
    take(s.b1, s.H);
    take(s.W2, (size_t)s.H * s.H);
    take(s.b2, s.H);
    take(s.W3, (size_t)s.K * s.H);
    take(s.b3, s.K);
    for (int q = 0; q < s.nL; q++)
        if (!(s.Ls[q] >= 1.f)) return set_error(ALTO_E_INVAL, "candidate segment counts must be >= 1");
    s.loaded = true;
    g_sel = std::move(s);
    return ALTO_OK;
}

int alto_select(const alto_tensor *t, int mode, int R, int prec, alto_exec *out) {
    if (!t || !out) return set_error(ALTO_E_INVAL, "null argument");
    if (mode < 0 || mode >= t->N) return set_error(ALTO_E_INVAL, "mode out of range");
    if (R < 1 || R > ALTO_MAX_RANK) return set_error(ALTO_E_INVAL, "R must be in 1..256");
    const int src = select_impl(t, mode, R, prec, out);
    if (src == kPlanOutside || src == kPlanClose) {
        // outside the training range, or close predictions: the plan found by
        // timing, once there is one
        const auto it = t->tuned.find(tuned_key(mode, R, prec));
        if (it != t->tuned.end()) *out = it->second;
    }
    return ALTO_OK;
}

}  // extern "C"
