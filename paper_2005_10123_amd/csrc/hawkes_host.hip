// hawkes_host.hip -- hawkes_host_eval: the log-likelihood, its gradient and the self-excitation
// probabilities on the host's CPU cores with SIMD vectorisation (the paper's multi-core CPU design,
// Section 2.3: rows partitioned over threads, each thread keeping its row's coordinates in registers
// and vectorising the loop over the other events, running sums only).  Host code only; a separate,
// explicitly requested evaluation, never a fallback of the device entry points.
//
// Binary64 throughout.  Per row i (events sorted by time), over all events j: the background term
// B = exp(-r^2/(2 tau_x^2) - dt^2/(2 tau_t^2)) and its moments r^2 B, dt^2 B; over the causal events
// j < c_i (t_j < t_i) the trigger term E = exp(-omega dt - r^2/(2 h^2)) and its moments dt E, r^2 E.
// Splitting each row's loop at c_i leaves two mask-free loops that vectorise.  Then lambda_i,
// Lambda_i, ell_i, pi_i and the gradient terms as in the device epilogue; totals summed in row
// order, so the result does not depend on the thread count.
#include "hawkes_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

namespace hawkes {
namespace {

// 2^a for a <= 0: a = k + f with k = round(a) (adding 1.5 * 2^52 rounds a to an integer, which
// then sits in the low bits of the sum's significand), |f| <= 1/2, the degree-10 polynomial
// minimising the maximal relative error of 2^f on [-1/2, 1/2] (the same Remez fit as the device's
// binary64 exponential, csrc/exp2_minimax.py), and 2^k written into the exponent field from the
// sum's bits with integer adds and shifts (no double-to-integer conversion, which has no vector
// form below AVX-512DQ).  Arguments below -1022 give 0 (the terms lost are below 2^-1022 of the
// diagonal term 1).  Branch-free, so the loops below vectorise.
inline double exp2_host(double a)
{
    const double big = 6755399441055744.0;  // 1.5 * 2^52, bit pattern 0x4338000000000000
    const double ac = a < -1022.0 ? -1022.0 : a;
    const double sum = ac + big;
    const double kd = sum - big;
    const double f = ac - kd;
    double p = 7.03735743919096230754e-09;
    p = p * f + 1.02085352821412315164e-07;
    p = p * f + 1.32156624055817323250e-06;
    p = p * f + 1.52526581335867644459e-05;
    p = p * f + 1.54035299619204323106e-04;
    p = p * f + 1.33335582285240734912e-03;
    p = p * f + 9.61812910803399277737e-03;
    p = p * f + 5.55041086644591438737e-02;
    p = p * f + 2.40226506959087704463e-01;
    p = p * f + 6.93147180559949727119e-01;
    p = p * f + 1.0;
    unsigned long long sb;
    std::memcpy(&sb, &sum, sizeof sb);
    const unsigned long long bits = (sb - 0x4338000000000000ULL + 1023ULL) << 52;  // (k + 1023) << 52
    double scale;
    std::memcpy(&scale, &bits, sizeof scale);
    return a < -1022.0 ? 0.0 : p * scale;
}

struct Coef {
    double nab, nbb, nae, nbe;  // negated base-2 exponent coefficients, as in the device pass
};

// Versions of the row loop for AVX-512, AVX2 + FMA (x86-64-v3) and the baseline, chosen at load
// time (host compilation only; the device pass never emits host functions).
#ifdef __HIP_DEVICE_COMPILE__
#define HAWKES_HOST_CLONES
#else
#define HAWKES_HOST_CLONES __attribute__((target_clones("avx512f", "arch=x86-64-v3", "default")))
#endif

// The six sums of one row: over j in [0, n) the background ones, over j in [0, c) the trigger ones.
HAWKES_HOST_CLONES void row_sums(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ t, int64_t n, int64_t c,
    double xi, double yi, double ti, Coef k, double* __restrict__ S)
{
    double sb = 0.0, sbr = 0.0, sbt = 0.0, se = 0.0, set = 0.0, ser = 0.0;
#pragma clang loop vectorize(enable) interleave(enable)
    for (int64_t j = 0; j < n; ++j) {
        const double dx = xi - x[j], dy = yi - y[j], dt = ti - t[j];
        const double r2 = dx * dx + dy * dy, dt2 = dt * dt;
        const double b = exp2_host(k.nab * r2 + k.nbb * dt2);
        sb += b;
        sbr += r2 * b;
        sbt += dt2 * b;
    }
#pragma clang loop vectorize(enable) interleave(enable)
    for (int64_t j = 0; j < c; ++j) {
        const double dx = xi - x[j], dy = yi - y[j], dt = ti - t[j];
        const double r2 = dx * dx + dy * dy;
        const double e = exp2_host(k.nae * r2 + k.nbe * dt);
        se += e;
        set += dt * e;
        ser += r2 * e;
    }
    S[0] = sb;
    S[1] = sbr;
    S[2] = sbt;
    S[3] = se;
    S[4] = set;
    S[5] = ser;
}

double normal_cdf(double z) { return 0.5 * std::erfc(-z * 0.70710678118654752440); }
double normal_pdf(double z) { return std::exp(-0.5 * z * z) * 0.39894228040143267794; }

}  // namespace
}  // namespace hawkes

using namespace hawkes;

extern "C" hawkes_status hawkes_host_eval(const double* x, const double* y, const double* t, int64_t n,
                                          const hawkes_params* p, int threads, double* out7, double* out_pi)
{
    if (!x || !y || !t || !out7) return fail(HAWKES_EINVAL, "NULL pointer argument");
    if (n < 1) return fail(HAWKES_EINVAL, "n = %lld < 1", (long long)n);
    hawkes_status st = check_params(p);
    if (st != HAWKES_OK) return st;
    for (int64_t k = 0; k < n; ++k) {
        if (!std::isfinite(x[k]) || !std::isfinite(y[k]) || !std::isfinite(t[k]))
            return fail(HAWKES_EINVAL, "event %lld has a non-finite coordinate", (long long)k);
        if (t[k] < 0.0) return fail(HAWKES_EINVAL, "event %lld has t = %g < 0", (long long)k, t[k]);
    }
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    threads = (int)std::min<int64_t>(threads, n);

    // Events sorted by (t, input index); c_i = #{j : t_j < t_i}.
    std::vector<int64_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return t[a] < t[b]; });
    std::vector<double> xs(n), ys(n), ts(n);
    std::vector<int64_t> cut(n);
    for (int64_t k = 0; k < n; ++k) {
        xs[k] = x[perm[k]];
        ys[k] = y[perm[k]];
        ts[k] = t[perm[k]];
        cut[k] = (k > 0 && ts[k] == ts[k - 1]) ? cut[k - 1] : k;
    }
    const double T = ts[n - 1];
    const double log2e = 1.44269504088896340736, two_pi = 6.28318530717958647693;
    const double mu0 = p->mu0, tx = p->tau_x, tt = p->tau_t, th = p->theta, om = p->omega, h = p->h;
    const Coef k{-log2e / (2.0 * tx * tx), -log2e / (2.0 * tt * tt), -log2e / (2.0 * h * h), -log2e * om};
    const double cb = mu0 / (std::pow(two_pi, 1.5) * tx * tx * tt);
    const double ce = th * om / (two_pi * h * h);

    // Per-row results (ell_i, gradient terms, pi_i), rows dealt to the threads in interleaved chunks
    // (later rows have longer trigger loops).
    std::vector<double> row((size_t)n * 8);
    constexpr int64_t kChunkRows = 64;
    auto work = [&](int w) {
        for (int64_t r0 = (int64_t)w * kChunkRows; r0 < n; r0 += (int64_t)threads * kChunkRows) {
            for (int64_t i = r0; i < std::min(n, r0 + kChunkRows); ++i) {
                double S[6];
                row_sums(xs.data(), ys.data(), ts.data(), n, cut[i], xs[i], ys[i], ts[i], k, S);
                const double ti = ts[i], u = T - ti;
                const double lam = cb * S[0] + ce * S[3];
                const double bg_int = normal_cdf(u / tt) - normal_cdf(-ti / tt);
                const double Lam = mu0 * bg_int - th * std::expm1(-om * u);
                const double inv = 1.0 / lam;
                const double k2pih2 = 1.0 / (two_pi * h * h);
                double* o = row.data() + (size_t)i * 8;
                o[0] = std::log(lam) - Lam;
                o[1] = cb * S[0] / mu0 * inv - bg_int;
                o[2] = cb * (-2.0 * S[0] / tx + S[1] / (tx * tx * tx)) * inv;
                o[3] = cb * (-S[0] / tt + S[2] / (tt * tt * tt)) * inv +
                       (mu0 / (tt * tt)) * (u * normal_pdf(u / tt) + ti * normal_pdf(ti / tt));
                o[4] = om * k2pih2 * S[3] * inv + std::expm1(-om * u);
                o[5] = th * k2pih2 * (S[3] - om * S[4]) * inv - th * u * std::exp(-om * u);
                o[6] = ce * (-2.0 * S[3] / h + S[5] / (h * h * h)) * inv;
                o[7] = ce * S[3] * inv;
            }
        }
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < threads; ++w) pool.emplace_back(work, w);
    work(0);
    for (auto& th_ : pool) th_.join();

    for (int q = 0; q < 7; ++q) out7[q] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int q = 0; q < 7; ++q) out7[q] += row[(size_t)i * 8 + q];
    if (out_pi)
        for (int64_t i = 0; i < n; ++i) out_pi[perm[i]] = row[(size_t)i * 8 + 7];
    return HAWKES_OK;
}
