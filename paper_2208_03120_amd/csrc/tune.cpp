// Measured cost table of the fast-summation autotuner (Sec. 5 parameters).
//
// The tuner's candidates trade window taps against grid size: a larger oversampled grid n
// admits a smaller cutoff m for the same window error, so spreading and interpolation get
// cheaper while the fold and the FFT passes grow.  The exchange rate between the two is
// measured here on the device instead of assumed: calibration plans with fixed parameters
// on synthetic uniform points are created through the public plan calls and their
// launches timed with mot_plan_profile.
#include <chrono>
#include <cmath>
#include <vector>

#include "host.h"

using mot::kTuneM;
using mot::kTuneN;

namespace {

constexpr int kPointN = 1 << 15;  // points per marginal of the point-cost plans
constexpr int kGridK = 17;        // marginals of the grid-cost star (16 edges)
constexpr int kGridN = 256;       // points per marginal of the grid-cost star
constexpr int kProfileSweeps = 3;

// splitmix64: uniform doubles in [0, 1)
struct Rng {
    uint64_t s;
    double next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    }
};

// K marginals of n uniform points in [-1/4, 1/4)^d with uniform-random normalised weights.
void synth(int K, int d, int n, uint64_t seed, std::vector<double> &pts, std::vector<double> &w)
{
    Rng r{seed};
    pts.resize((size_t)K * n * d);
    w.resize((size_t)K * n);
    for (auto &x : pts) x = 0.5 * r.next() - 0.25;
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += (w[(size_t)k * n + i] = 0.5 + r.next());
        for (int i = 0; i < n; ++i) w[(size_t)k * n + i] /= s;
    }
}

// Mean per-sweep milliseconds of the launches whose kind is in `kinds` (one sweep
// first, untimed, so that one-time costs stay out).
int timed_kinds(mot_plan P, std::initializer_list<int> kinds, double *ms, mot_plan_info *info)
{
    int32_t done = 0;
    double S = 0, err = 0;
    MOT_TRY(mot_sinkhorn(P, 1, 0.0, 0.0, 0, &done, &S, &err));
    std::vector<mot_step_timing> t(4096);
    const int nt = mot_plan_profile(P, kProfileSweeps, t.data(), (int32_t)t.size());
    if (nt < 0) return nt;
    double sum = 0.0;
    for (int i = 0; i < nt; ++i)
        for (int k : kinds)
            if (t[i].kind == k) sum += t[i].ms_mean;
    *ms = sum;
    return mot_plan_get_info(P, info);
}

int measure(mot_tune_table *T)
{
    std::vector<double> pts, w;
    // point costs: a two-marginal path, both products spread and interpolate kPointN points
    for (int d = 1; d <= 3; ++d) {
        synth(2, d, kPointN, 0x5eed0000ULL + d, pts, w);
        const int64_t n[2] = {kPointN, kPointN};
        const int32_t parent[2] = {-1, 0};
        const int grid = d == 1 ? 256 : (d == 2 ? 128 : 64);
        for (int m = 2; m < 2 + kTuneM; ++m) {
            mot_fastsum_params fs{};
            fs.M = 8;
            fs.n = grid;
            fs.m = m;
            fs.p = 4;
            mot_plan P = nullptr;
            MOT_TRY(mot_plan_create(&P, 2, d, n, pts.data(), w.data(), MOT_TREE, parent, 0.05, MOT_NFFT,
                                    MOT_PREC_MIXED, &fs, MOT_HOST, nullptr, nullptr));
            double ms = 0.0;
            mot_plan_info info{};
            const int rc = timed_kinds(P, {2, 5}, &ms, &info);
            mot_plan_destroy(P);
            if (rc < 0) return rc;
            T->point_ns[d - 1][m - 2] = ms * 1e6 / (2.0 * kPointN);
        }
    }
    // grid costs: a star whose 32 products share every fold and FFT launch
    for (int d = 1; d <= 3; ++d) {
        synth(kGridK, d, kGridN, 0x6e1d0000ULL + d, pts, w);
        std::vector<int64_t> n(kGridK, kGridN);
        std::vector<int32_t> parent(kGridK, 0);
        parent[0] = -1;
        // largest grid first: a grid too small for any box of the cloud (n = 16: the tile edge
        // 17 - 2m leaves no room for the window halo) is never a tuner candidate, and its
        // entry repeats the next grid's cost per box cell
        for (int k = kTuneN - 1; k >= 0; --k) {
            mot_fastsum_params fs{};
            fs.n = 16 << k;
            fs.M = fs.n / 4;
            fs.m = 4;
            fs.p = 4;
            mot_plan P = nullptr;
            const int cr = mot_plan_create(&P, kGridK, d, n.data(), pts.data(), w.data(), MOT_TREE, parent.data(),
                                           0.05, MOT_NFFT, MOT_PREC_MIXED, &fs, MOT_HOST, nullptr, nullptr);
            if (cr == MOT_EDOMAIN && k + 1 < kTuneN) {
                T->grid_us[d - 1][k] = T->grid_us[d - 1][k + 1];
                T->box_cells[d - 1][k] = T->box_cells[d - 1][k + 1];
                continue;
            }
            MOT_TRY(cr);
            double ms = 0.0;
            mot_plan_info info{};
            const int rc = timed_kinds(P, {3, 4}, &ms, &info);
            mot_plan_destroy(P);
            if (rc < 0) return rc;
            double box = 1.0;
            for (int c = 0; c < d; ++c) box *= info.box_len[c];
            T->grid_us[d - 1][k] = ms * 1e3 / (2.0 * (kGridK - 1));
            T->box_cells[d - 1][k] = box;
        }
    }
    return MOT_OK;
}

}  // namespace

extern "C" {

int mot_tune_measure(mot_tune_table *out)
{
    if (!out) return MOT_EINVAL;
    mot_tune_table T{};
    MOT_HIP(hipGetDevice(&T.device));
    const auto t0 = std::chrono::steady_clock::now();
    MOT_TRY(measure(&T));
    T.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    T.measured = 1;
    *out = T;
    return MOT_OK;
}

int mot_tune_install(const mot_tune_table *table) { return mot::install_tune_table(table); }

int mot_tune_resolve(int32_t d, double eta, double half_width, int64_t n_max, const mot_fastsum_params *fs,
                     mot_fastsum_params *out, double *est_err)
{
    if (!out || d < 1 || d > 3 || !(eta > 0) || !(half_width > 0) || n_max < 1) return MOT_EINVAL;
    mot::Extent E;
    for (int c = 0; c < d; ++c) {
        E.lo[c] = -half_width;
        E.hi[c] = half_width;
    }
    E.width_max = 2.0 * half_width;
    E.diag = 2.0 * half_width * std::sqrt((double)d);
    mot::NfftParams Q;
    MOT_TRY(mot::resolve_params(d, eta, E, fs, n_max, &Q));
    mot_fastsum_params r{};
    r.M = Q.M;
    r.n = Q.n;
    r.m = Q.m;
    r.p = Q.p;
    r.tau = Q.tau;
    r.eps_B = Q.eps_B;
    r.tile = Q.T;
    r.chunk = Q.chunk;
    r.target_rel_err = fs && fs->target_rel_err > 0 ? fs->target_rel_err : 1e-7;
    *out = r;
    if (est_err) *est_err = Q.est_err;
    return MOT_OK;
}

}  // extern "C"
