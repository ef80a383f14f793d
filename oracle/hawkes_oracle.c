/*
 * hawkes_oracle.c -- plain FP64 reference evaluator of the spatiotemporal Hawkes
 * log-likelihood, its gradient and the self-excitation probabilities.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this file;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg do.  It shares no
 * code, header or constant with the GPU library.  Built with
 *     gcc -O2 -fno-fast-math -ffp-contract=off -shared -fPIC hawkes_oracle.c -lm
 * so every operation is an IEEE binary64 round-to-nearest operation in source order and every
 * transcendental is libm's.
 *
 * What is computed (arXiv 2005.10123, Section 2.1 "Model", the log-likelihood equation):
 *
 *   lambda_n = sum_{n'=1..N} mu0 / (tau_x^2 tau_t) * phi2((x_n - x_n')/tau_x) * phi1((t_n - t_n')/tau_t)
 *            + sum_{n': t_n' < t_n} theta * omega / h^2 * exp(-omega (t_n - t_n')) * phi2((x_n - x_n')/h)
 *   Lambda_n = mu0 * (Phi((T - t_n)/tau_t) - Phi(-t_n/tau_t)) - theta * (exp(-omega (T - t_n)) - 1)
 *   ell      = sum_n [ log lambda_n - Lambda_n ],      T = max_n t_n
 *
 * with phi1(v) = exp(-v^2/2)/sqrt(2 pi), phi2(u) = exp(-|u|^2/2)/(2 pi) (d = 2) and Phi the
 * standard normal CDF.  Readings taken where the paper is garbled or silent:
 *   - the excitation coefficient is theta*omega/h^d: the printed theta/(omega h^d) contradicts the
 *     paper's own closed-form integral, whose temporal part integrates theta*omega*exp(-omega s);
 *   - the background sum includes n' = n, exactly as printed (so lambda_n >= its own KDE term > 0);
 *   - the background time kernel is two-sided (later events count), as printed;
 *   - the excitation indicator is the strict t_n' < t_n (ties excluded), as printed;
 *   - the observation window is [0, T] in time with no spatial edge correction, as printed.
 *
 * The gradient (the paper gives none) is the exact derivative of ell in the natural coordinates
 * Theta = (mu0, tau_x, tau_t, theta, omega, h).  Writing B = the unnormalised background kernel,
 * E = the unnormalised excitation kernel, r2 = |x_n - x_n'|^2, dt = t_n - t_n', u = T - t_n,
 * c_b = mu0 (2 pi)^(-3/2) tau_x^-2 tau_t^-1 and c_e = theta omega (2 pi)^-1 h^-2:
 *   d lambda/d mu0   = c_b Sb / mu0
 *   d lambda/d tau_x = c_b (-2 Sb / tau_x + Sbr / tau_x^3)
 *   d lambda/d tau_t = c_b (-Sb / tau_t + Sbt / tau_t^3)
 *   d lambda/d theta = omega / (2 pi h^2) * Se
 *   d lambda/d omega = theta / (2 pi h^2) * (Se - omega Set)
 *   d lambda/d h     = c_e (-2 Se / h + Ser / h^3)
 *   d Lambda/d mu0   = Phi(u/tau_t) - Phi(-t/tau_t)
 *   d Lambda/d tau_t = -(mu0/tau_t^2) (u phi1(u/tau_t) + t phi1(t/tau_t))
 *   d Lambda/d theta = -(exp(-omega u) - 1)
 *   d Lambda/d omega = theta u exp(-omega u)
 * where Sb = sum B, Sbr = sum r2 B, Sbt = sum dt^2 B, Se = sum E, Set = sum dt E, Ser = sum r2 E.
 *
 * The self-excitation probability (the paper's probability equation) is pi_n = xi_n / lambda_n with
 * xi_n the excitation part of lambda_n.
 *
 * Pins (what fixes this file against the paper and the mathematics, in tests/):
 *   closed form at N = 1; library probability densities (scipy.stats) and 40-digit mpmath sums on
 *   small inputs; quadrature of the intensity against Lambda; central finite differences against
 *   the gradient; the identity mu0 dl/dmu0 + theta dl/dtheta = N - Lambda; theta = 0 and all-ties
 *   invariants; permutation and translation invariance; planted mutants that each pin must catch.
 */
#include <math.h>
#include <stddef.h>

static const double ORACLE_TWO_PI = 6.28318530717958647692528676655900577;

static double norm_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

static double norm_pdf(double z) { return exp(-0.5 * z * z) / sqrt(ORACLE_TWO_PI); }

/* Per-row quantities of one event n against all N events. */
typedef struct {
    double lambda, Lambda, ell, pi;
    double grad[6];
    double sums[6]; /* Sb, Sbr, Sbt, Se, Set, Ser */
} oracle_row;

static double max_time(const double* t, long n)
{
    double T = t[0];
    for (long k = 1; k < n; ++k)
        if (t[k] > T) T = t[k];
    return T;
}

static void oracle_one_row(const double* x, const double* y, const double* t, long n, double T,
                           const double* th, long i, oracle_row* out)
{
    const double mu0 = th[0], tx = th[1], tt = th[2], theta = th[3], omega = th[4], h = th[5];
    const double cb = mu0 / (pow(ORACLE_TWO_PI, 1.5) * tx * tx * tt);
    const double ce = theta * omega / (ORACLE_TWO_PI * h * h);

    double Sb = 0.0, Sbr = 0.0, Sbt = 0.0, Se = 0.0, Set = 0.0, Ser = 0.0;
    for (long j = 0; j < n; ++j) {
        const double dx = x[i] - x[j];
        const double dy = y[i] - y[j];
        const double dt = t[i] - t[j];
        const double r2 = dx * dx + dy * dy;
        const double b = exp(-r2 / (2.0 * tx * tx) - dt * dt / (2.0 * tt * tt));
        Sb += b;
        Sbr += r2 * b;
        Sbt += dt * dt * b;
        if (t[j] < t[i]) {
            const double e = exp(-omega * dt - r2 / (2.0 * h * h));
            Se += e;
            Set += dt * e;
            Ser += r2 * e;
        }
    }

    const double lambda = cb * Sb + ce * Se;
    const double u = T - t[i];
    const double Lambda = mu0 * (norm_cdf(u / tt) - norm_cdf(-t[i] / tt)) - theta * expm1(-omega * u);

    const double dlam[6] = {
        cb * Sb / mu0,
        cb * (-2.0 * Sb / tx + Sbr / (tx * tx * tx)),
        cb * (-Sb / tt + Sbt / (tt * tt * tt)),
        omega / (ORACLE_TWO_PI * h * h) * Se,
        theta / (ORACLE_TWO_PI * h * h) * (Se - omega * Set),
        ce * (-2.0 * Se / h + Ser / (h * h * h)),
    };
    const double dLam[6] = {
        norm_cdf(u / tt) - norm_cdf(-t[i] / tt),
        0.0,
        -(mu0 / (tt * tt)) * (u * norm_pdf(u / tt) + t[i] * norm_pdf(t[i] / tt)),
        -expm1(-omega * u),
        theta * u * exp(-omega * u),
        0.0,
    };

    out->lambda = lambda;
    out->Lambda = Lambda;
    out->ell = log(lambda) - Lambda;
    out->pi = ce * Se / lambda;
    for (int p = 0; p < 6; ++p) out->grad[p] = dlam[p] / lambda - dLam[p];
    out->sums[0] = Sb;
    out->sums[1] = Sbr;
    out->sums[2] = Sbt;
    out->sums[3] = Se;
    out->sums[4] = Set;
    out->sums[5] = Ser;
}

/*
 * Whole log-likelihood and gradient.
 *   x, y, t   : n events in any order (host memory, read only)
 *   th        : 6 parameters (mu0, tau_x, tau_t, theta, omega, h)
 *   out       : 7 doubles: ell, then d ell / d Theta in the order of th
 *   row_ell, row_Lambda, row_pi : n doubles each or NULL
 *   row_grad  : n*6 doubles (row-major, 6 per event) or NULL
 * Returns 0, or -1 when n < 1 or a required pointer is NULL.  Performs no other validation.
 */
int hawkes_oracle_eval(const double* x, const double* y, const double* t, long n, const double* th,
                       double* out, double* row_ell, double* row_Lambda, double* row_pi,
                       double* row_grad)
{
    if (n < 1 || !x || !y || !t || !th || !out) return -1;
    const double T = max_time(t, n);
    double ell = 0.0, grad[6] = {0, 0, 0, 0, 0, 0};
    for (long i = 0; i < n; ++i) {
        oracle_row r;
        oracle_one_row(x, y, t, n, T, th, i, &r);
        ell += r.ell;
        for (int p = 0; p < 6; ++p) grad[p] += r.grad[p];
        if (row_ell) row_ell[i] = r.ell;
        if (row_Lambda) row_Lambda[i] = r.Lambda;
        if (row_pi) row_pi[i] = r.pi;
        if (row_grad)
            for (int p = 0; p < 6; ++p) row_grad[i * 6 + p] = r.grad[p];
    }
    out[0] = ell;
    for (int p = 0; p < 6; ++p) out[1 + p] = grad[p];
    return 0;
}

/*
 * Selected rows only, each against all n events (for sampled checks at sizes where the full
 * double loop would take too long).  For every k < nrows, row rows[k] writes 16 doubles at
 * out + 16 k: lambda, Lambda, ell, pi, grad[6], Sb, Sbr, Sbt, Se, Set, Ser.
 * Returns 0, or -1 on n < 1, a NULL pointer or a row index outside [0, n).
 */
int hawkes_oracle_rows(const double* x, const double* y, const double* t, long n, const double* th,
                       const long* rows, long nrows, double* out)
{
    if (n < 1 || !x || !y || !t || !th || (nrows > 0 && (!rows || !out))) return -1;
    for (long k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= n) return -1;
    const double T = max_time(t, n);
    for (long k = 0; k < nrows; ++k) {
        oracle_row r;
        oracle_one_row(x, y, t, n, T, th, rows[k], &r);
        double* o = out + 16 * k;
        o[0] = r.lambda;
        o[1] = r.Lambda;
        o[2] = r.ell;
        o[3] = r.pi;
        for (int p = 0; p < 6; ++p) o[4 + p] = r.grad[p];
        for (int p = 0; p < 6; ++p) o[10 + p] = r.sums[p];
    }
    return 0;
}
