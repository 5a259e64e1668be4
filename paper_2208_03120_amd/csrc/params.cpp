// Fast-summation parameters: the regularised kernel, its Fourier coefficients, the
// window transform, the spectral multiplier and the autotuner.  Host FP64.
//
// Sec. 5 (eqs. Ker-reg, kappa_tilde, fourier_serie, fft) builds a 2 tau-periodic,
// p times differentiable kernel that equals exp(-|x|^2/eta) on |x| <= tau - eps_B, and
// approximates it by 2M Fourier coefficients per dimension.  Reading of the boundary
// polynomial: kappa_B has degree 2p, its derivatives 0..p match kappa at tau - eps_B and
// its derivatives 1..p vanish at tau (this reproduces the worked example of Fig. 1).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "host.h"

namespace mot {

// d^r/dx^r exp(-x^2/eta) for r = 0..rmax via Hermite polynomials:
// d^r/dt^r exp(-t^2) = (-1)^r H_r(t) exp(-t^2), t = x / sqrt(eta).
static void kappa_derivs(double x, double eta, int rmax, double *out)
{
    const double t = x / std::sqrt(eta), e = std::exp(-t * t);
    double hm1 = 0.0, h = 1.0;
    for (int r = 0; r <= rmax; ++r) {
        out[r] = ((r & 1) ? -1.0 : 1.0) * h * e * std::pow(eta, -0.5 * r);
        const double hn = 2.0 * t * h - 2.0 * r * hm1;
        hm1 = h;
        h = hn;
    }
}

// Coefficients q_j of kappa_B(x) = sum_j q_j (x - a)^j, a = tau - eps_B (degree 2p).
void kappa_B_shifted(double eta, double tau, double eps_B, int p, std::vector<double> &q)
{
    const int n = 2 * p + 1;
    std::vector<double> A((size_t)n * n, 0.0), rhs(n, 0.0), der(p + 1);
    const double a = tau - eps_B;
    kappa_derivs(a, eta, p, der.data());
    int row = 0;
    for (int r = 0; r <= p; ++r, ++row) {  // derivative r at x = a: r! q_r
        double f = 1.0;
        for (int i = 2; i <= r; ++i) f *= i;
        A[(size_t)row * n + r] = f;
        rhs[row] = der[r];
    }
    for (int r = 1; r <= p; ++r, ++row) {  // derivative r at x = tau vanishes
        for (int j = r; j < n; ++j) {
            double f = 1.0;
            for (int i = j - r + 1; i <= j; ++i) f *= i;  // j! / (j-r)!
            A[(size_t)row * n + j] = f * std::pow(eps_B, j - r);
        }
        rhs[row] = 0.0;
    }
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)c * n + j], A[(size_t)piv * n + j]);
            std::swap(rhs[c], rhs[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[(size_t)r * n + c] / A[(size_t)c * n + c];
            for (int j = c; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
            rhs[r] -= f * rhs[c];
        }
    }
    q.assign(n, 0.0);
    for (int r = n - 1; r >= 0; --r) {
        double s = rhs[r];
        for (int j = r + 1; j < n; ++j) s -= A[(size_t)r * n + j] * q[j];
        q[r] = s / A[(size_t)r * n + r];
    }
}

// Regularised radial kernel, eq. (Ker-reg).
double kappa_R(double r, double eta, double tau, double eps_B, const std::vector<double> &q)
{
    r = std::fabs(r);
    const double a = tau - eps_B;
    if (r <= a) return std::exp(-r * r / eta);
    const double x = std::min(r, tau) - a;
    double v = 0.0;
    for (int j = (int)q.size() - 1; j >= 0; --j) v = v * x + q[j];
    return v;
}

// kappa_hat(k) for k_c in 0..M (it is even in every coordinate), eq. (fft):
//   (2M)^-d sum_{x in (tau/M){-M..M-1}^d} kappa_tilde(x) prod_c cos(pi k_c x_c / tau).
// Output index ((k0 * (M+1)) + k1) * (M+1) + k2.
void kappa_hat_even(int d, int M, double eta, double tau, double eps_B, int p,
                    std::vector<double> &khat)
{
    std::vector<double> q;
    kappa_B_shifted(eta, tau, eps_B, p, q);
    const int S = 2 * M, H = M + 1;
    std::vector<double> C((size_t)H * S);
    for (int k = 0; k < H; ++k)
        for (int j = 0; j < S; ++j) C[(size_t)k * S + j] = std::cos(M_PI * k * (double)(j - M) / M);
    // samples
    size_t ns = 1;
    for (int c = 0; c < d; ++c) ns *= S;
    std::vector<double> cur(ns);
    for (size_t idx = 0; idx < ns; ++idx) {
        size_t rem = idx;
        double r2 = 0.0;
        for (int c = d - 1; c >= 0; --c) {
            const int j = (int)(rem % S);
            rem /= S;
            const double x = tau * (double)(j - M) / M;
            r2 += x * x;
        }
        cur[idx] = kappa_R(std::sqrt(r2), eta, tau, eps_B, q);
    }
    // transform one axis at a time: shape (outer, S, inner) -> (outer, H, inner)
    std::vector<int> dims(d, S);
    for (int ax = 0; ax < d; ++ax) {
        size_t outer = 1, inner = 1;
        for (int c = 0; c < ax; ++c) outer *= dims[c];
        for (int c = ax + 1; c < d; ++c) inner *= dims[c];
        std::vector<double> nxt(outer * H * inner, 0.0);
        for (size_t o = 0; o < outer; ++o)
            for (int k = 0; k < H; ++k) {
                double *dst = &nxt[(o * H + k) * inner];
                for (int j = 0; j < S; ++j) {
                    const double w = C[(size_t)k * S + j];
                    const double *src = &cur[(o * S + j) * inner];
                    for (size_t i = 0; i < inner; ++i) dst[i] += w * src[i];
                }
            }
        dims[ax] = H;
        cur.swap(nxt);
    }
    const double norm = std::pow(2.0 * M, -d);
    for (double &v : cur) v *= norm;
    khat.swap(cur);
}

// Modified Bessel function I0 by its power series (arguments up to ~80 here).
static double bessel_i0(double x)
{
    const double y = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int j = 1; j < 500; ++j) {
        term *= y / ((double)j * j);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// Fourier transform of the normalised window psi(s)/psi(0) at frequency k (grid
// units): Psi(k) = I0(m sqrt(b^2 - w^2)) * pi m / sinh(b m), w = 2 pi k / n.
double kb_fourier(double k, const NfftParams &P)
{
    const double w = 2.0 * M_PI * k / P.n, b = P.kb_b, m = P.m;
    const double z = m * std::sqrt(std::max(b * b - w * w, 0.0));
    return bessel_i0(z) * M_PI * m / std::sinh(b * m);
}

// Spectral multiplier on the half spectrum (last axis k >= 0):
//   D(k) = kappa_hat(k) w(k) / prod_c Psi(k_c)^2,  |k_c| <= M,
// w(k) = (1[k in B] + 1[-k in B]) / 2 with B = {-M..M-1}^d: taking the real part of the
// sum over the asymmetric index set B equals summing the symmetrised coefficients.
// Layout: d=3 [k2 0..M][k1+M][k0+M], d=2 [k1 0..M][k0+M], d=1 [k0 0..M].
void build_multiplier(int d, const NfftParams &P, double eta, std::vector<float> &D)
{
    const int M = P.M, H = M + 1, B = 2 * M + 1;
    std::vector<double> kh;
    kappa_hat_even(d, M, eta, P.tau, P.eps_B, P.p, kh);
    std::vector<double> psi2(H);
    for (int k = 0; k < H; ++k) {
        const double v = kb_fourier(k, P);
        psi2[k] = v * v;
    }
    auto weight = [&](const int *k) {
        bool inB = true, negB = true;
        for (int c = 0; c < d; ++c) {
            if (k[c] == M) inB = false;
            if (k[c] == -M) negB = false;
        }
        return 0.5 * ((inB ? 1.0 : 0.0) + (negB ? 1.0 : 0.0));
    };
    auto khat = [&](const int *k) {
        size_t idx = 0;
        for (int c = 0; c < d; ++c) idx = idx * H + (size_t)std::abs(k[c]);
        return kh[idx];
    };
    if (d == 1) {
        D.resize(H);
        for (int k0 = 0; k0 <= M; ++k0) {
            const int k[1] = {k0};
            D[k0] = (float)(khat(k) * weight(k) / psi2[k0]);
        }
    } else if (d == 2) {
        D.resize((size_t)H * B);
        for (int k1 = 0; k1 <= M; ++k1)
            for (int k0 = -M; k0 <= M; ++k0) {
                const int k[2] = {k0, k1};
                D[(size_t)k1 * B + (k0 + M)] =
                    (float)(khat(k) * weight(k) / (psi2[std::abs(k0)] * psi2[k1]));
            }
    } else {
        D.resize((size_t)H * B * B);
        for (int k2 = 0; k2 <= M; ++k2)
            for (int k1 = -M; k1 <= M; ++k1)
                for (int k0 = -M; k0 <= M; ++k0) {
                    const int k[3] = {k0, k1, k2};
                    D[((size_t)k2 * B + (k1 + M)) * B + (k0 + M)] = (float)(
                        khat(k) * weight(k) / (psi2[std::abs(k0)] * psi2[std::abs(k1)] * psi2[k2]));
                }
    }
}

void build_twiddle(int n, std::vector<float2> &tw)
{
    tw.resize(n / 2);
    for (int k = 0; k < n / 2; ++k) {
        const double a = 2.0 * M_PI * k / n;
        tw[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
}

// Active box and tiles.  Cells of a coordinate x are floor(x s + o); the box spans the
// patches (T + 2m - 1 cells starting at tile * T - m + 1) of every tile holding a point.
int build_box(int d, const Extent &ext, NfftParams *P)
{
    P->s = P->n / (2.0 * P->tau);
    for (int c = 0; c < 3; ++c) {
        P->o[c] = 0.0;
        P->lo[c] = 0;
        P->L[c] = 1;
        P->ntile[c] = 1;
        P->tmin[c] = 0;
    }
    for (int c = 0; c < d; ++c) {
        P->o[c] = 0.5 * P->n - ext.ctr[c] * P->s;
        const double ulo = ext.lo[c] * P->s + P->o[c], uhi = ext.hi[c] * P->s + P->o[c];
        const int clo = (int)std::floor(ulo), chi = (int)std::floor(uhi);
        const int tlo = clo / P->T, thi = chi / P->T;
        if (clo < 0) return MOT_EDOMAIN;
        P->tmin[c] = tlo;
        P->ntile[c] = thi - tlo + 1;
        P->lo[c] = tlo * P->T - P->m + 1;
        P->L[c] = P->ntile[c] * P->T + 2 * P->m - 1;
        if (P->lo[c] < 0 || P->lo[c] + P->L[c] > P->n) return MOT_EDOMAIN;
    }
    P->W = P->T + 2 * P->m - 1;
    return MOT_OK;
}

// ---------------------------------------------------------------------------------------
// Autotuner.  Accuracy model for one product, relative to sum_j |v_j|:
//   Fourier part: the 1-D truncated series of the regularised kernel against kappa on
//   [0, diag] (evaluated exactly from the 1-D coefficients), times d;
//   window part: the Kaiser-Bessel aliasing bound 4 pi (sqrt(m) + m) (1 - 1/sigma)^(1/4)
//   exp(-2 pi m sqrt(1 - 1/sigma)).
// Cost model: spreading and interpolation touch (2m)^d cells per point; the pruned FFT
// costs about box^d log n.  The cheapest candidate meeting the target is chosen.
static double fourier_err_1d(int M, double eta, double tau, double eps_B, int p, double diag)
{
    std::vector<double> kh;
    kappa_hat_even(1, M, eta, tau, eps_B, p, kh);
    double worst = 0.0;
    const int R = 96;
    for (int i = 0; i <= R; ++i) {
        const double r = diag * i / R;
        double s = kh[0];
        for (int k = 1; k < M; ++k) s += 2.0 * kh[k] * std::cos(M_PI * k * r / tau);
        s += kh[M] * std::cos(M_PI * M * r / tau);  // the unpaired -M term (real part)
        worst = std::max(worst, std::fabs(s - std::exp(-r * r / eta)));
    }
    return worst;
}

static double kb_err(int m, double sigma)
{
    const double a = std::sqrt(1.0 - 1.0 / sigma);
    return 4.0 * M_PI * (std::sqrt((double)m) + m) * std::pow(1.0 - 1.0 / sigma, 0.25) *
           std::exp(-2.0 * M_PI * m * a);
}

// Spreading and interpolation work on 16-cell patches: tiles of T = 17 - 2m cells.
static int tile_for(int m) { return 17 - 2 * m; }

// Cost of one product for a candidate: the measured table when one is installed, else the
// analytic model (window taps of the points plus the box's line transforms).
static std::mutex g_tune_mu;
static mot_tune_table g_tune{};  // measured == 0: analytic model

int install_tune_table(const mot_tune_table *t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!t) {
        g_tune = mot_tune_table{};
        return MOT_OK;
    }
    for (int d = 0; d < 3; ++d) {
        for (int m = 0; m < kTuneM; ++m)
            if (!(std::isfinite(t->point_ns[d][m]) && t->point_ns[d][m] > 0)) return MOT_EINVAL;
        for (int k = 0; k < kTuneN; ++k)
            if (!(std::isfinite(t->grid_us[d][k]) && t->grid_us[d][k] > 0 && std::isfinite(t->box_cells[d][k]) &&
                  t->box_cells[d][k] >= 1))
                return MOT_EINVAL;
    }
    g_tune = *t;
    g_tune.measured = 1;
    return MOT_OK;
}

static double product_cost(int d, int64_t n_max, int n, int m, double box)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tune.measured) {
            const int k = (int)std::lround(std::log2((double)n)) - 4;  // n = 16 << k
            const int mi = std::min(std::max(m - 2, 0), kTuneM - 1);
            return (double)n_max * g_tune.point_ns[d - 1][mi] * 1e-3 +
                   g_tune.grid_us[d - 1][k] * box / g_tune.box_cells[d - 1][k];
        }
    }
    return 2.0 * (double)n_max * std::pow(2.0 * m, d) + 10.0 * box * std::log2((double)n) * d;
}

int resolve_params(int d, double eta, const Extent &ext, const mot_fastsum_params *fs,
                   int64_t n_max, NfftParams *out, double eta_hi)
{
    mot_fastsum_params F{};
    if (fs) F = *fs;
    if (F.m < 0 || F.m > kMaxTaps / 2 || F.M < 0 || F.n < 0 || F.p < 0 || F.tile < 0 || F.chunk < 0)
        return MOT_EINVAL;
    if (F.n > 0 && (F.n < kMinN || F.n > kMaxN || (F.n & (F.n - 1)) != 0)) return MOT_EINVAL;
    if (F.M > 0 && F.n > 0 && 2 * F.M >= F.n) return MOT_EINVAL;
    if (F.tile > 0 && F.m > 0 && F.tile != tile_for(F.m)) return MOT_EINVAL;
    const double target = F.target_rel_err > 0 ? F.target_rel_err : 1e-7;
    const double diag = std::max(ext.diag, 1e-12);
    NfftParams best;
    double best_cost = -1.0;
    std::vector<int> p_list = F.p > 0 ? std::vector<int>{F.p} : std::vector<int>{3, 4, 5};
    std::vector<double> eb_list;
    if (F.eps_B > 0)
        eb_list.push_back(F.eps_B);
    else
        for (double f : {0.05, 0.1, 0.15, 0.25, 0.4, 0.6}) eb_list.push_back(f * diag);
    std::vector<int> M_list;
    if (F.M > 0)
        M_list.push_back(F.M);
    else
        for (int M : {4, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64, 80, 96, 112, 127})
            M_list.push_back(M);
    for (int p : p_list)
        for (double eb : eb_list) {
            double tau = F.tau > 0 ? F.tau : (diag + eb) * (1.0 + 1e-9);
            if (tau <= eb + ext.diag) return MOT_EDOMAIN;
            int Mfound = -1;
            double ferr = 0.0;
            for (int M : M_list) {
                ferr = d * fourier_err_1d(M, eta, tau, eb, p, ext.diag);
                if (eta_hi > eta) ferr = std::max(ferr, d * fourier_err_1d(M, eta_hi, tau, eb, p, ext.diag));
                if (F.M > 0 || ferr <= 0.5 * target) {
                    Mfound = M;
                    break;
                }
            }
            if (Mfound < 0) continue;
            // grid sizes: powers of two with oversampling sigma = n / (2M) > 1
            std::vector<int> n_list;
            if (F.n > 0)
                n_list.push_back(F.n);
            else
                for (int n = kMinN; n <= kMaxN; n *= 2)
                    if (n >= 3 * Mfound) n_list.push_back(n);
            for (int n : n_list) {
                if (n <= 2 * Mfound || n > kMaxN || n < kMinN) continue;
                const double sigma = n / (2.0 * Mfound);
                int m = F.m;
                if (m <= 0) {
                    for (m = 2; m <= 8; ++m)
                        if (kb_err(m, sigma) <= 0.5 * target) break;
                    if (m > 8) continue;
                }
                NfftParams P;
                P.M = Mfound;
                P.n = n;
                P.m = m;
                P.p = p;
                P.tau = tau;
                P.eps_B = eb;
                P.sigma = sigma;
                P.T = tile_for(m);
                if (build_box(d, ext, &P) != MOT_OK) continue;
                P.kb_b = M_PI * (2.0 - 1.0 / sigma);
                double box = 1.0;
                for (int c = 0; c < d; ++c) box *= P.L[c];
                const double cost = product_cost(d, n_max, n, m, box);
                if (best_cost < 0 || cost < best_cost) {
                    best_cost = cost;
                    best = P;
                    best.est_err = ferr + kb_err(m, sigma);
                }
            }
        }
    if (best_cost < 0) return MOT_EDOMAIN;
    int chunk = F.chunk > 0 ? F.chunk : (d == 3 ? 512 : 2048);
    best.chunk = chunk;
    *out = best;
    return MOT_OK;
}

// ---------------------------------------------------------------------------------------
// Truncated path.  Dropping the source terms with exp(-r^2 / eta) < eps changes a product
// by at most eps sum_j v_j.  For a uniform cloud of bounding-box volume V, a target at a
// corner of the box sums about (pi eta)^(d/2) / (2^d V) of the total source weight, so
// eps = target (pi eta)^(d/2) / (2^d V) keeps the relative error of such products near
// the target.  The cell side h = r_c / q is chosen by a cost model of the kernel: one
// wavefront per item of at most 64 R targets from a run of B consecutive cells of a row,
// scanning the rows of cells whose box distance to the run is at most r_c.
int64_t trunc_cells(int d, const TruncParams &T)
{
    int64_t c = 1;
    for (int k = 0; k < d; ++k) c *= T.nc;
    return c;
}

int trunc_row_range(int d, const TruncParams &T, const int cc[3], int B, int ri, int64_t *row_base,
                    int *xa, int *xb)
{
    const int w = T.w, span = 2 * w + 1;
    int del[2] = {0, 0};
    if (d == 3) {
        del[0] = ri / span - w;
        del[1] = ri % span - w;
    } else if (d == 2) {
        del[0] = ri - w;
    }
    double used = 0.0;
    int64_t base = 0;
    for (int c = 0; c < d - 1; ++c) {
        const int x = cc[c] + del[c];
        if (x < 0 || x >= T.nc) return 0;
        const int e = std::abs(del[c]) - 1;
        if (e > 0) used += (double)e * e;
        base = base * T.nc + x;
    }
    const double rem = T.q2 - used;
    if (rem < 0.0) return 0;
    const int wl = std::min(w, 1 + (int)std::floor(std::sqrt(rem)));
    *row_base = base * T.nc;
    *xa = std::max(cc[d - 1] - wl, 0);
    *xb = std::min(cc[d - 1] + B - 1 + wl, T.nc - 1);
    return 1;
}

// E[ceil(X / cap)] for a Poisson count X with mean lam (pmf in log space).
static double expected_chunks(double lam, int cap)
{
    if (lam <= 0.0) return 0.0;
    if (lam > 1e4) return lam / cap + 0.5;  // concentrated: ceil adds half an item on average
    const double sd = std::sqrt(lam);
    const int k0 = std::max(0, (int)std::floor(lam - 12.0 * sd - 5.0));
    const int k1 = (int)std::ceil(lam + 12.0 * sd + 20.0);
    double s = 0.0;
    for (int k = std::max(k0, 1); k <= k1; ++k)
        s += std::exp(k * std::log(lam) - lam - std::lgamma(k + 1.0)) * std::ceil((double)k / cap);
    return s;
}

// Modelled wave cycles of one product: per row ~100, per 64-source stage ~200, per source
// and target slot ~40 (FP32 coordinate differences) or ~66 (FP64 exponent).  Points are
// taken as Poisson counts per cell: lam_t / lam_s targets / sources per full cell (the
// cloud's density times h^d).  A run of B cells holding k targets takes ceil(k / 64R)
// items; the runs are those of the cells covering the cloud's box.
double trunc_cost(int d, const TruncParams &T, double lam_t, double lam_s, int B, int R, bool wide)
{
    const int span = 2 * T.w + 1;
    const int rows_total = d == 1 ? 1 : (d == 2 ? span : span * span);
    TruncParams U = T;
    U.nc = 1 << 20;  // no clipping at the grid edge
    const int cc[3] = {1 << 19, 1 << 19, 1 << 19};
    double cells = 0.0, rows = 0.0;
    for (int ri = 0; ri < rows_total; ++ri) {
        int64_t base;
        int xa, xb;
        if (!trunc_row_range(d, U, cc, B, ri, &base, &xa, &xb)) continue;
        rows += 1.0;
        cells += xb - xa + 1;
    }
    double runs = 1.0;
    for (int c = 0; c < d - 1; ++c) runs *= T.box_cells[c];
    runs *= std::ceil(T.box_cells[d - 1] / B);
    const double items = runs * expected_chunks(lam_t * B, 64 * R);
    const double src = cells * lam_s;
    return items * (rows * 100.0 + (src / 64.0 + rows) * 200.0 + src * R * (wide ? 66.0 : 40.0));
}

// sqrt(log2(e) / eta) times the half-diagonal of a run of B cells: the largest scaled
// coordinate of a target relative to the run's centre.  The FP32 form is used up to 3.
static double run_extent(int d, const TruncParams &T, double sch, int B)
{
    return sch * std::sqrt(0.25 * B * B + 0.25 * (d - 1));
}

void trunc_choose_run(int d, const TruncParams &T, double lam_t, double lam_s, int max_r, double sch, bool fp64,
                      int *B, int *R, int *wide)
{
    double best = -1.0;
    *B = 1;
    *R = 1;
    *wide = 0;
    for (int b : {1, 2, 3, 4, 6, 8, 12, 16}) {
        if (b > T.nc) break;
        for (int r : {1, 2, 4}) {
            if (r > max_r) break;
            for (int w = 0; w < 2; ++w) {
                if (!fp64 && w == 0 && run_extent(d, T, sch, b) > 3.0) continue;
                const double c = trunc_cost(d, T, lam_t, lam_s, b, r, fp64 || w == 1);
                if (best < 0 || c < best) {
                    best = c;
                    *B = b;
                    *R = r;
                    *wide = fp64 ? 0 : w;
                }
            }
        }
    }
}

int resolve_trunc(int d, double eta, const Extent &ext, const mot_fastsum_params *fs, double n_mean,
                  TruncParams *out)
{
    const double target = fs && fs->target_rel_err > 0 ? fs->target_rel_err : 1e-7;
    if (!(target < 1.0)) return MOT_EINVAL;
    const double g0 = std::sqrt(M_PI * eta);
    double V = 1.0;
    for (int c = 0; c < d; ++c) V *= std::max(ext.hi[c] - ext.lo[c], g0);
    const double frac = std::pow(M_PI * eta, 0.5 * d) / (std::pow(2.0, d) * V);
    TruncParams T;
    T.eps = target * std::min(1.0, frac);
    T.rc = std::sqrt(eta * std::log(1.0 / T.eps));
    T.est_err = target;
    for (int c = 0; c < 3; ++c) T.glo[c] = c < d ? ext.lo[c] : 0.0;
    const int nc_max = d == 1 ? (1 << 20) : (d == 2 ? 2048 : 128);
    double best = -1.0;
    for (double q : {0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 8.0}) {
        TruncParams C = T;
        C.h = T.rc / q;
        const double ncd = std::floor(ext.width_max / C.h) + 1.0;
        if (ncd > nc_max) continue;
        C.nc = (int)ncd;
        C.q2 = q * q * (1.0 + 1e-6);
        C.w = 1 + (int)std::floor(std::sqrt(C.q2));
        {
            const int span = 2 * C.w + 1;
            if ((d == 3 ? span * span : (d == 2 ? span : 1)) > kMaxTruncRows) continue;
        }
        double Vb = 1.0;
        for (int c = 0; c < d; ++c) {
            const double wc = std::max(ext.hi[c] - ext.lo[c], C.h);
            C.box_cells[c] = wc / C.h;
            Vb *= wc;
        }
        const double lam = std::max(n_mean, 1.0) * std::pow(C.h, d) / Vb;  // points per full cell
        const double sch = std::sqrt(1.4426950408889634 / eta) * C.h;
        int wide = 0;
        trunc_choose_run(d, C, lam, lam, 4, sch, false, &C.B, &C.R, &wide);
        const double cost = trunc_cost(d, C, lam, lam, C.B, C.R, wide != 0);
        if (best < 0 || cost < best) {
            best = cost;
            *out = C;
        }
    }
    if (best < 0) return MOT_EDOMAIN;
    return MOT_OK;
}

}  // namespace mot
