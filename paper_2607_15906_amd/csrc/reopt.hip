// ADAPT with every angle re-optimised after each appended operator (textbook
// ADAPT, Sec. II.B), on the device.
//
// The ansatz state is the chain of layers psi(theta) = L_k ... L_1 psi_0, each
// layer the substepped O(5) Taylor propagator of Eq. 5-6 of one pool
// generator, L(theta) = T5(theta / s)^s, with s = max(1, ceil(max(|theta|, pi)
// ||A||_1 / 0.5)) so that the energy is smooth in the angles.  One evaluation
// of the energy and its gradient is
//   * the forward pass: k pair launches, every intermediate state kept;
//   * sigma = H psi_k and E (the energy launches of the one-shot calls);
//   * the backward pass: k pair launches from lam = sigma - E psi_k, each
//     adding its layer's Re <lam | dL phi> per block and applying L^+ to lam;
//   * one copy of the per-block partials and the energy back to the host,
//     where the gradient 2 sum / <psi|psi> is summed in a fixed order.
// BFGS runs on the host over these evaluations, the screen (Eq. 4) and the
// selection run on the optimised state.

#include <cmath>
#include <string>
#include <vector>

#include "runtime.h"

namespace gocp {
namespace {

constexpr double kBfgsC1 = 1e-4;       // sufficient decrease
constexpr double kBfgsFtol = 1e-14;    // rounding allowance of E in that test (relative)
constexpr int kBfgsHalvings = 30;
constexpr double kTieRtol = 1e-12;     // selection tie band (as the frozen path)

struct Reopt {
    gocp_ctx *ctx = nullptr;
    const Ham *h = nullptr;
    const Pool *p = nullptr;
    const DevicePool *dp = nullptr;
    int dtype = 0, nq = 0, npb = 1;
    size_t dim = 0, es = 16;
    char *mem = nullptr;          // forward states, lam, sigma, partials
    char *F = nullptr;
    double2 *lam = nullptr, *sigma = nullptr;
    double *partial = nullptr;
    double *hpart = nullptr;      // pinned: partials, then the state record
    std::vector<int> ops;
    int evals = 0;

    ~Reopt() {
        if (mem) (void)hipFree(mem);
        if (hpart) (void)hipHostFree(hpart);
    }
    void *state(int i) { return F + (size_t)i * dim * es; }
    int substeps(int j, double th) const {
        return std::max(1, (int)std::ceil(std::max(std::fabs(th), M_PI) * p->op_norm1[j] / 0.5));
    }
    void forward(const std::vector<double> &th) {
        hipStream_t s = ctx->user_stream;
        for (size_t i = 0; i < ops.size(); ++i) {
            const int ns = substeps(ops[i], th[i]);
            launch_layer_fwd(dtype, state((int)i), state((int)i + 1), dp->pop, dp->pterm, ops[i], ns, th[i] / ns, nq, s);
        }
    }
    // E(theta) and its gradient; the forward states stay in F.
    double eval(const std::vector<double> &th, std::vector<double> &g) {
        hipStream_t s = ctx->user_stream;
        const int k = (int)ops.size();
        forward(th);
        const AdaptState *st = enqueue_energy_sigma(ctx, h, state(k), dtype, sigma);
        for (int i = k - 1; i >= 0; --i) {
            const int ns = substeps(ops[i], th[i]);
            launch_layer_adj(dtype, state(i), lam, partial + (size_t)i * npb, dp->pop, dp->pterm, ops[i], ns, th[i] / ns,
                             nq, i == k - 1 ? sigma : nullptr, state(k), st, s);
        }
        AdaptState hs;
        hip_check(hipMemcpyAsync(hpart, partial, sizeof(double) * k * npb, hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        ++evals;
        if (hs.status || !(hs.nrm > 0.0) || !std::isfinite(hs.energy))
            throw Error(GOCP_ENUMERIC, "non-finite energy or zero norm during re-optimisation");
        g.assign(k, 0.0);
        for (int i = 0; i < k; ++i) {
            double a = 0.0;
            for (int b = 0; b < npb; ++b) a += hpart[(size_t)i * npb + b];
            g[i] = 2.0 * a / hs.nrm;
            if (!std::isfinite(g[i])) throw Error(GOCP_ENUMERIC, "non-finite gradient during re-optimisation");
        }
        return hs.energy;
    }
};

double dot(const std::vector<double> &a, const std::vector<double> &b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

double max_abs(const std::vector<double> &a) {
    double m = 0.0;
    for (double v : a) m = std::max(m, std::fabs(v));
    return m;
}

// BFGS, inverse-Hessian form: direction -Hinv g (reset to -g when it is not a
// descent direction), backtracking from step 1 by halving until sufficient
// decrease (up to the rounding of E), the update skipped when s.y is not
// positive enough; stops at max |g| < gtol, after maxiter steps or when the
// line search fails.  Returns the steps taken; x, f, g hold the result.
int bfgs(Reopt &R, std::vector<double> &x, double &f, std::vector<double> &g, double gtol, int maxiter) {
    const size_t n = x.size();
    f = R.eval(x, g);
    std::vector<double> hinv(n * n, 0.0), p(n), xn(n), gn, sv(n), yv(n), tmp(n * n);
    for (size_t i = 0; i < n; ++i) hinv[i * n + i] = 1.0;
    int it = 0;
    while (it < maxiter && max_abs(g) >= gtol) {
        for (size_t i = 0; i < n; ++i) {
            double a = 0.0;
            for (size_t j = 0; j < n; ++j) a += hinv[i * n + j] * g[j];
            p[i] = -a;
        }
        double gp = dot(g, p);
        if (!(gp < 0.0)) {
            std::fill(hinv.begin(), hinv.end(), 0.0);
            for (size_t i = 0; i < n; ++i) {
                hinv[i * n + i] = 1.0;
                p[i] = -g[i];
            }
            gp = dot(g, p);
        }
        double t = 1.0, fn = 0.0;
        bool ok = false;
        for (int k = 0; k <= kBfgsHalvings; ++k) {
            for (size_t i = 0; i < n; ++i) xn[i] = x[i] + t * p[i];
            fn = R.eval(xn, gn);
            if (fn <= f + kBfgsC1 * t * gp + kBfgsFtol * (1.0 + std::fabs(f))) {
                ok = true;
                break;
            }
            t *= 0.5;
        }
        if (!ok) break;
        for (size_t i = 0; i < n; ++i) {
            sv[i] = xn[i] - x[i];
            yv[i] = gn[i] - g[i];
        }
        const double sy = dot(sv, yv);
        if (sy > 1e-12 * std::sqrt(dot(sv, sv)) * std::sqrt(dot(yv, yv))) {
            // Hinv <- (I - rho s y^T) Hinv (I - rho y s^T) + rho s s^T
            const double rho = 1.0 / sy;
            for (size_t i = 0; i < n; ++i)          // tmp = (I - rho s y^T) Hinv
                for (size_t j = 0; j < n; ++j) {
                    double a = 0.0;
                    for (size_t l = 0; l < n; ++l) a += ((i == l ? 1.0 : 0.0) - rho * sv[i] * yv[l]) * hinv[l * n + j];
                    tmp[i * n + j] = a;
                }
            for (size_t i = 0; i < n; ++i)          // Hinv = tmp (I - rho y s^T) + rho s s^T
                for (size_t j = 0; j < n; ++j) {
                    double a = 0.0;
                    for (size_t l = 0; l < n; ++l) a += tmp[i * n + l] * ((l == j ? 1.0 : 0.0) - rho * yv[l] * sv[j]);
                    hinv[i * n + j] = a + rho * sv[i] * sv[j];
                }
        }
        x = xn;
        f = fn;
        g = gn;
        ++it;
    }
    return it;
}

}  // namespace
}  // namespace gocp

using namespace gocp;

extern "C" {

int adapt_reopt_solve(gocp_ctx *ctx, const gocp_ham *hh, const gocp_pool *pp, void *psi_dev, int dtype,
                      const gocp_reopt_params *params, gocp_reopt_result *res) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    check_dtype(dtype);
    if (!params || !res || !psi_dev) throw Error(GOCP_EINVAL, "null params, result or state");
    if (!res->energies || !res->ops || !res->thetas || !res->gnorms) throw Error(GOCP_EINVAL, "null result arrays");
    const Ham *h = as_ham(hh);
    const Pool *p = as_pool(pp);
    if (h->n_qubits != p->n_qubits) throw Error(GOCP_ESHAPE, "Hamiltonian and pool act on different qubit counts");
    const int max_iter = params->max_iter;
    if (max_iter < 0) throw Error(GOCP_EINVAL, "negative max_iter");
    const double gtol = params->bfgs_gtol > 0.0 ? params->bfgs_gtol : 1e-8;
    const int bmax = params->bfgs_max_iter > 0 ? params->bfgs_max_iter : 200;
    Reopt R;
    R.ctx = ctx;
    R.h = h;
    R.p = p;
    R.dtype = dtype;
    R.nq = h->n_qubits;
    R.dim = (size_t)1 << R.nq;
    R.es = dtype == GOCP_C64 ? 8 : 16;
    R.npb = (int)std::max<size_t>(1, (R.dim / 2 + kPairBlock - 1) / kPairBlock);
    R.dp = device_pool(*p, ctx->device);
    device_ham(*h, ctx->device);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t fb = al((size_t)(max_iter + 1) * R.dim * R.es), lb = al(R.dim * 16);
    const size_t pb = al(sizeof(double) * std::max(max_iter, 1) * R.npb);
    hip_check(hipMalloc(&R.mem, fb + 2 * lb + pb), "hipMalloc re-optimisation workspace");
    R.F = R.mem;
    R.lam = reinterpret_cast<double2 *>(R.mem + fb);
    R.sigma = reinterpret_cast<double2 *>(R.mem + fb + lb);
    R.partial = reinterpret_cast<double *>(R.mem + fb + 2 * lb);
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&R.hpart), pb, 0), "hipHostMalloc");
    hipStream_t s = ctx->user_stream;
    hip_check(hipMemcpyAsync(R.state(0), psi_dev, R.dim * R.es, hipMemcpyDeviceToDevice, s), "D2D");

    const int M = p->n_ops();
    std::vector<double> g(M), theta, grad;
    int n_iter = 0, converged = 0;
    for (int it = 0;; ++it) {
        // screen and energy of the current state (psi_0 or the optimised one)
        const int k = (int)R.ops.size();
        const AdaptState *st = enqueue_energy_sigma(ctx, h, R.state(k), dtype, R.sigma);
        AdaptState hs;
        hip_check(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (hs.status || !(hs.nrm > 0.0)) throw Error(GOCP_ENUMERIC, "non-finite energy or zero norm");
        res->energies[it] = hs.energy;
        if (it >= max_iter) break;
        const int rc = pool_gradients(ctx, hh, pp, R.state(k), dtype, g.data(), 0);
        if (rc != GOCP_OK) throw Error(rc, std::string("gradient screen: ") + gocp_last_error());
        double gmax = 0.0, sq = 0.0;
        for (int j = 0; j < M; ++j) {
            gmax = std::max(gmax, std::fabs(g[j]));
            sq += g[j] * g[j];
        }
        int jsel = 0;
        for (int j = 0; j < M; ++j)
            if (std::fabs(g[j]) >= gmax * (1.0 - kTieRtol)) {
                jsel = j;
                break;
            }
        const double gn = std::sqrt(sq);
        res->gnorms[it] = gn;
        if (gn < params->grad_tol) {
            converged = 1;
            break;
        }
        R.ops.push_back(jsel);
        theta.push_back(0.0);
        double f = 0.0;
        const int steps = bfgs(R, theta, f, grad, gtol, bmax);
        R.forward(theta);                      // the state at the returned angles
        res->ops[it] = jsel;
        if (res->bfgs_steps) res->bfgs_steps[it] = steps;
        if (res->bfgs_evals) res->bfgs_evals[it] = R.evals;
        R.evals = 0;
        n_iter = it + 1;
    }
    for (int i = 0; i < n_iter; ++i) res->thetas[i] = theta[i];
    res->n_iter = n_iter;
    res->converged = converged;
    // the optimised state, normalised, back into psi_dev
    const AdaptState *st = enqueue_energy_sigma(ctx, h, R.state(n_iter), dtype, R.sigma);
    AdaptState hs;
    hip_check(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    launch_scale_copy(dtype, R.state(n_iter), psi_dev, (uint32_t)R.dim, 1.0 / std::sqrt(hs.nrm), s);
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    return GOCP_OK;
    GOCP_GUARD_END
}

}  // extern "C"
