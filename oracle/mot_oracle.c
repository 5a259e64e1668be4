/*
 * Plain FP64 CPU oracle for tree- and circle-structured entropic multi-marginal
 * optimal transport (Ba & Quellmalz, "Accelerating the Sinkhorn algorithm for
 * sparse multi-marginal optimal transport by fast Fourier transforms").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library is
 * checked against.  It shares no code, header, table or helper with the GPU
 * path and must never be linked into it.  Only tests/, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.
 *
 * Everything is double precision, written for clarity rather than speed:
 *   - kernel products are the plain definition (Sec. 5, eq. fastsum-sum),
 *     summed over sources in ascending index order;
 *   - the tree solver follows Algorithm 2 step by step (Sec. 4.1);
 *   - the circle solver follows Algorithm 3 step by step (Sec. 4.2), with the
 *     dense matrix products written as plain loops;
 *   - point binning is the plain definition used by the GPU library
 *     (cell = floor(x*s + o), clamped; tile = cell / T; stable sort by tile).
 * OpenMP only splits independent output rows across threads; each output
 * element is accumulated sequentially, so results do not depend on the thread
 * count.
 *
 * Points of marginal k are rows [off[k], off[k+1]) of a row-major (N_total x d)
 * array; weights and scaling vectors are concatenated the same way.  Marginal
 * indices are 0-based here (the paper's marginal 1 is index 0).
 *
 * Compile with -ffp-contract=off: the binning must not fuse x*s+o into an FMA.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_MAXITER 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)
#define ORC_ENUMERIC (-6)

/* ------------------------------------------------------------------------ */
/* Gaussian kernel product, Sec. 5 eq. (fastsum-sum) with the kernel matrix of
 * Sec. 4 eq. (K-matrix):
 *   out[i] = sum_j v[j] * exp(-|xt_i - xs_j|^2 / eta),  j ascending.          */
void orc_kernel_apply(int d, long nt, const double *xt, long ns, const double *xs,
                      const double *v, double eta, double *out)
{
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nt; ++i) {
        double acc = 0.0;
        for (long j = 0; j < ns; ++j) {
            double dist2 = 0.0;
            for (int c = 0; c < d; ++c) {
                double diff = xt[i * d + c] - xs[j * d + c];
                dist2 += diff * diff;
            }
            acc += v[j] * exp(-dist2 / eta);
        }
        out[i] = acc;
    }
}

/* Dense kernel matrix K^{(a,b)}[i][j] = exp(-|x^a_i - x^b_j|^2/eta), row-major. */
static void kernel_matrix(int d, long na, const double *xa, long nb, const double *xb,
                          double eta, double *Kab)
{
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < na; ++i)
        for (long j = 0; j < nb; ++j) {
            double dist2 = 0.0;
            for (int c = 0; c < d; ++c) {
                double diff = xa[i * d + c] - xb[j * d + c];
                dist2 += diff * diff;
            }
            Kab[i * nb + j] = exp(-dist2 / eta);
        }
}

/* ------------------------------------------------------------------------ */
/* Tree structure, Sec. 4.1.  parent[0] = -1 (root), parent[k] < k otherwise. */

typedef struct {
    int K, d;
    const long *off;
    const double *pts;
    const int *parent;
    double eta;
    double **beta;  /* beta[k] (k >= 1) has length n_{p(k)}: alpha^{(p(k),k)} */
    double **gamma; /* gamma[k] has length n_k: alpha^{(k,p(k))}, gamma[0] = 1  */
    double *work;   /* scratch vector of length max n_k                        */
    const double *edge_w; /* NULL or [K]: weight w_k of the edge {p(k), k}, Sec. 6.2 */
    const int *free_node; /* NULL or [K]: nonzero = no marginal constraint at k    */
} tree_t;

/* The edge {p(k), k} has cost w_k |x - y|^2 (eq. cost_function_barycenter_tree), so its
 * kernel is exp(-|x - y|^2 / (eta / w_k)). */
static double edge_eta(const tree_t *T, int k) { return T->edge_w ? T->eta / T->edge_w[k] : T->eta; }
static int is_free(const tree_t *T, int k) { return T->free_node && T->free_node[k]; }

static long tn(const tree_t *T, int k) { return T->off[k + 1] - T->off[k]; }
static const double *tpts(const tree_t *T, int k) { return T->pts + T->off[k] * T->d; }

/* out = prod_{t in C_k, t != skip} beta_t  (ascending t), length n_k.
 * The empty product is the all-ones vector, eq. (comp_wise_multi_beta_tree). */
static void child_product(const tree_t *T, int k, int skip, double *out)
{
    long n = tn(T, k);
    for (long i = 0; i < n; ++i) out[i] = 1.0;
    for (int t = k + 1; t < T->K; ++t) {
        if (T->parent[t] != k || t == skip) continue;
        for (long i = 0; i < n; ++i) out[i] *= T->beta[t][i];
    }
}

/* beta_k = K^{(p(k),k)} (phi^k (.) beta^{(.)C_k}), Algorithm 2 step 4. */
static void compute_beta(tree_t *T, const double *const *phi, int k)
{
    int p = T->parent[k];
    long nk = tn(T, k);
    child_product(T, k, -1, T->work);
    for (long i = 0; i < nk; ++i) T->work[i] = phi[k][i] * T->work[i];
    orc_kernel_apply(T->d, tn(T, p), tpts(T, p), nk, tpts(T, k), T->work, edge_eta(T, k),
                     T->beta[k]);
}

/* gamma_k = K^{(p(k),k)T} (phi^{p} (.) gamma_p (.) beta^{(.)C_p \ k}), eq. (gamma_tree). */
static void compute_gamma(tree_t *T, const double *const *phi, int k)
{
    if (k == 0) {
        for (long i = 0; i < tn(T, 0); ++i) T->gamma[0][i] = 1.0;
        return;
    }
    int p = T->parent[k];
    long np_ = tn(T, p);
    child_product(T, p, k, T->work);
    for (long i = 0; i < np_; ++i) T->work[i] = (phi[p][i] * T->gamma[p][i]) * T->work[i];
    orc_kernel_apply(T->d, tn(T, k), tpts(T, k), np_, tpts(T, p), T->work, edge_eta(T, k),
                     T->gamma[k]);
}

static int tree_alloc(tree_t *T)
{
    if (T->K < 2) return ORC_EINVAL;
    long nmax = 0;
    for (int k = 0; k < T->K; ++k)
        if (tn(T, k) > nmax) nmax = tn(T, k);
    T->beta = (double **)calloc((unsigned)T->K, sizeof(double *));
    T->gamma = (double **)calloc((unsigned)T->K, sizeof(double *));
    T->work = (double *)malloc((size_t)nmax * sizeof(double));
    if (!T->beta || !T->gamma || !T->work) return ORC_ENOMEM;
    for (int k = 0; k < T->K; ++k) {
        T->gamma[k] = (double *)malloc((size_t)tn(T, k) * sizeof(double));
        if (!T->gamma[k]) return ORC_ENOMEM;
        if (k > 0) {
            T->beta[k] = (double *)malloc((size_t)tn(T, T->parent[k]) * sizeof(double));
            if (!T->beta[k]) return ORC_ENOMEM;
        }
    }
    return ORC_OK;
}

static void tree_free(tree_t *T)
{
    for (int k = 0; k < T->K; ++k) {
        if (T->beta) free(T->beta[k]);
        if (T->gamma) free(T->gamma[k]);
    }
    free(T->beta);
    free(T->gamma);
    free(T->work);
}

static int tree_check(int K, const int *parent)
{
    if (K < 2 || parent[0] != -1) return ORC_EINVAL;
    for (int k = 1; k < K; ++k)
        if (parent[k] < 0 || parent[k] >= k) return ORC_EINVAL;
    return ORC_OK;
}

/* Sinkhorn for tree structure, Algorithm 2.
 *   phi    in: initial scaling vectors (phi^(0)); out: the last computed ones.
 *   S_hist receives S^(r) for every completed sweep r (length >= max_sweeps).
 * Stops when |S^(r) - S^(r-1)| < delta (delta > 0) or after max_sweeps sweeps.
 * Generalised barycenters (Sec. 6.2): edge_w (NULL = all 1) weights the edge costs and
 * free_node (NULL = none) marks nodes without a marginal constraint; their phi is 1 in
 * every sweep (the modified update of the phi step) and their mu is not read.  The root
 * must be constrained: its update is the one that fixes the common scale of the
 * scalings, and without it the stale sibling messages of Algorithm 2 oscillate (two
 * children) or grow geometrically (more). */
int orc_tree_sinkhorn_ex(int K, int d, const long *off, const double *pts, const double *mu,
                         const int *parent, const double *edge_w, const int *free_node, double eta,
                         int max_sweeps, double delta, double *phi_cat, double *S_hist,
                         int *sweeps_done)
{
    if (tree_check(K, parent) != ORC_OK || eta <= 0.0 || d < 1) return ORC_EINVAL;
    if (edge_w)
        for (int k = 1; k < K; ++k)
            if (!(edge_w[k] > 0.0)) return ORC_EINVAL;
    if (free_node && free_node[0]) return ORC_EINVAL;
    tree_t T = {K, d, off, pts, parent, eta, NULL, NULL, NULL, edge_w, free_node};
    int rc = tree_alloc(&T);
    double **phi = (double **)malloc((size_t)K * sizeof(double *));
    double *phi_old = (double *)malloc((size_t)off[K] * sizeof(double));
    if (rc != ORC_OK || !phi || !phi_old) {
        tree_free(&T);
        free(phi);
        free(phi_old);
        return ORC_ENOMEM;
    }
    for (int k = 0; k < K; ++k) phi[k] = phi_cat + off[k];

    /* Initial upward pass, k = K..2 in the paper's numbering. */
    for (int k = K - 1; k >= 1; --k) compute_beta(&T, (const double *const *)phi, k);

    rc = ORC_MAXITER;
    int r;
    for (r = 0; r < max_sweeps; ++r) {
        memcpy(phi_old, phi_cat, (size_t)off[K] * sizeof(double));
        /* Downward pass: gamma_k and the new phi^k, k = 1..K. */
        for (int k = 0; k < K; ++k) {
            compute_gamma(&T, (const double *const *)phi, k);
            long nk = tn(&T, k);
            child_product(&T, k, -1, T.work);
            const double *muk = mu + off[k];
            for (long i = 0; i < nk; ++i)
                phi[k][i] = is_free(&T, k) ? 1.0 : muk[i] / (T.gamma[k][i] * T.work[i]);
        }
        /* Upward pass with the new phi, k = K..2. */
        for (int k = K - 1; k >= 1; --k) compute_beta(&T, (const double *const *)phi, k);

        /* S^(r) = eta (sum_k mu^k . log phi^k(r) - (mu^1 / phi^1(r+1)) . phi^1(r)).
         * Terms with mu = 0 contribute nothing (0 log 0 := 0); free nodes have none. */
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < K; ++k) {
            if (is_free(&T, k)) continue;
            for (long i = off[k]; i < off[k + 1]; ++i)
                if (mu[i] > 0.0) s1 += mu[i] * log(phi_old[i]);
        }
        for (long i = 0; i < tn(&T, 0); ++i)
            if (mu[i] > 0.0) s2 += (mu[i] / phi[0][i]) * phi_old[i];
        S_hist[r] = eta * (s1 - s2);

        for (long i = 0; i < off[K]; ++i)
            if (!isfinite(phi_cat[i])) {
                rc = ORC_ENUMERIC;
                break;
            }
        if (rc == ORC_ENUMERIC) {
            ++r;
            break;
        }
        if (delta > 0.0 && r >= 1 && fabs(S_hist[r] - S_hist[r - 1]) < delta) {
            rc = ORC_OK;
            ++r;
            break;
        }
    }
    *sweeps_done = r;
    tree_free(&T);
    free(phi);
    free(phi_old);
    return rc;
}

int orc_tree_sinkhorn(int K, int d, const long *off, const double *pts, const double *mu,
                      const int *parent, double eta, int max_sweeps, double delta,
                      double *phi_cat, double *S_hist, int *sweeps_done)
{
    return orc_tree_sinkhorn_ex(K, d, off, pts, mu, parent, NULL, NULL, eta, max_sweeps, delta,
                                phi_cat, S_hist, sweeps_done);
}

int orc_tree_marginals_ex(int K, int d, const long *off, const double *pts, const int *parent,
                          const double *edge_w, double eta, const double *phi_cat, double *P)
{
    if (tree_check(K, parent) != ORC_OK || eta <= 0.0) return ORC_EINVAL;
    tree_t T = {K, d, off, pts, parent, eta, NULL, NULL, NULL, edge_w, NULL};
    if (tree_alloc(&T) != ORC_OK) {
        tree_free(&T);
        return ORC_ENOMEM;
    }
    const double **phi = (const double **)malloc((size_t)K * sizeof(double *));
    for (int k = 0; k < K; ++k) phi[k] = phi_cat + off[k];
    for (int k = K - 1; k >= 1; --k) compute_beta(&T, phi, k);
    for (int k = 0; k < K; ++k) compute_gamma(&T, phi, k);
    for (int k = 0; k < K; ++k) {
        long nk = tn(&T, k);
        child_product(&T, k, -1, T.work);
        for (long i = 0; i < nk; ++i) P[off[k] + i] = (phi[k][i] * T.gamma[k][i]) * T.work[i];
    }
    free(phi);
    tree_free(&T);
    return ORC_OK;
}

int orc_tree_marginals(int K, int d, const long *off, const double *pts, const int *parent,
                       double eta, const double *phi_cat, double *P)
{
    return orc_tree_marginals_ex(K, d, off, pts, parent, NULL, eta, phi_cat, P);
}

/* ------------------------------------------------------------------------ */
/* Circle structure, Sec. 4.2.  Edges {k, k+1} and {K, 1}.                   */

typedef struct {
    int K, d;
    const long *off;
    const double *pts;
    double eta;
    double **Kedge; /* Kedge[k] = K^{(k,k+1 mod K)}, n_k x n_{k+1}            */
    double **beta;  /* beta[k] = alpha^{(k,1)}, n_k x n_1, k = 1..K-1 (0-based) */
    double *gam;    /* current gamma_k = lambda^{(1,k)}, n_1 x n_k             */
    double *gam_next;
    const double *closing; /* NULL or n_1 x d: the points sigma(x^1) that marginal 1 takes
                              on the closing edge {K, 1} (generalised Euler flows, Sec. 6.3) */
} circ_t;

static long cn(const circ_t *C, int k) { return C->off[k + 1] - C->off[k]; }
static const double *cpts(const circ_t *C, int k) { return C->pts + C->off[k] * C->d; }

/* beta_k = K^{(k,k+1)} (phi^{k+1} (.) beta_{k+1}), with beta_K = K^{(K,1)}
 * (Algorithm 3 step 4).  (.) of a vector and a matrix scales the rows. */
static void circ_beta(circ_t *C, const double *const *phi, int k)
{
    long n1 = cn(C, 0), nk = cn(C, k);
    if (k == C->K - 1) {
        memcpy(C->beta[k], C->Kedge[k], (size_t)(nk * n1) * sizeof(double));
        return;
    }
    long nk1 = cn(C, k + 1);
    const double *Kk = C->Kedge[k];
    const double *b1 = C->beta[k + 1];
    const double *ph = phi[k + 1];
    double *out = C->beta[k];
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nk; ++i) {
        double *row = out + i * n1;
        for (long j = 0; j < n1; ++j) row[j] = 0.0;
        for (long l = 0; l < nk1; ++l) {
            double a = Kk[i * nk1 + l] * ph[l];
            const double *brow = b1 + l * n1;
            for (long j = 0; j < n1; ++j) row[j] += a * brow[j];
        }
    }
}

/* gamma_k = gamma_{k-1} (phi^{k-1} (.) K^{(k-1,k)}), gamma_2 = K^{(1,2)}
 * (Algorithm 3 step 9, the lambda recursion of Theorem 4.3). Result in gam_next. */
static void circ_gamma_step(circ_t *C, const double *const *phi, int k)
{
    long n1 = cn(C, 0), nkm = cn(C, k - 1), nk = cn(C, k);
    const double *Kk = C->Kedge[k - 1];
    const double *ph = phi[k - 1];
    const double *g = C->gam;
    double *out = C->gam_next;
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n1; ++i) {
        double *row = out + i * nk;
        for (long j = 0; j < nk; ++j) row[j] = 0.0;
        for (long l = 0; l < nkm; ++l) {
            double a = g[i * nkm + l] * ph[l];
            const double *krow = Kk + l * nk;
            for (long j = 0; j < nk; ++j) row[j] += a * krow[j];
        }
    }
}

/* Row-wise inner product <G, H> with G = beta_k (n_k x n_1) and
 * H = (phi^1 (.) gamma_k)^T:  out[i] = sum_j beta_k[i][j] phi^1_j gamma_k[j][i]. */
static void circ_inner_beta_gamma(const circ_t *C, const double *const *phi, int k,
                                  const double *gk, double *out)
{
    long n1 = cn(C, 0), nk = cn(C, k);
    const double *bk = C->beta[k];
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nk; ++i) {
        double acc = 0.0;
        for (long j = 0; j < n1; ++j) acc += bk[i * n1 + j] * (phi[0][j] * gk[j * nk + i]);
        out[i] = acc;
    }
}

/* <K^{(1,2)}, (phi^2 (.) beta_2)^T>_i = sum_j K^{(1,2)}[i][j] phi^2_j beta_2[j][i]. */
static void circ_inner_root(const circ_t *C, const double *const *phi, double *out)
{
    long n1 = cn(C, 0), n2 = cn(C, 1);
    const double *K12 = C->Kedge[0];
    const double *b2 = C->beta[1];
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n1; ++i) {
        double acc = 0.0;
        for (long j = 0; j < n2; ++j) acc += K12[i * n2 + j] * (phi[1][j] * b2[j * n1 + i]);
        out[i] = acc;
    }
}

static int circ_alloc(circ_t *C)
{
    long n1 = cn(C, 0), nmax = 0;
    for (int k = 0; k < C->K; ++k)
        if (cn(C, k) > nmax) nmax = cn(C, k);
    C->Kedge = (double **)calloc((size_t)C->K, sizeof(double *));
    C->beta = (double **)calloc((size_t)C->K, sizeof(double *));
    C->gam = (double *)malloc((size_t)(n1 * nmax) * sizeof(double));
    C->gam_next = (double *)malloc((size_t)(n1 * nmax) * sizeof(double));
    if (!C->Kedge || !C->beta || !C->gam || !C->gam_next) return ORC_ENOMEM;
    for (int k = 0; k < C->K; ++k) {
        int k1 = (k + 1) % C->K;
        C->Kedge[k] = (double *)malloc((size_t)(cn(C, k) * cn(C, k1)) * sizeof(double));
        if (!C->Kedge[k]) return ORC_ENOMEM;
        /* the closing edge compares x^K with sigma(x^1) when a map is given */
        const double *xb = (k1 == 0 && C->closing) ? C->closing : cpts(C, k1);
        kernel_matrix(C->d, cn(C, k), cpts(C, k), cn(C, k1), xb, C->eta, C->Kedge[k]);
        if (k >= 1) {
            C->beta[k] = (double *)malloc((size_t)(cn(C, k) * n1) * sizeof(double));
            if (!C->beta[k]) return ORC_ENOMEM;
        }
    }
    return ORC_OK;
}

static void circ_free(circ_t *C)
{
    for (int k = 0; k < C->K; ++k) {
        if (C->Kedge) free(C->Kedge[k]);
        if (C->beta) free(C->beta[k]);
    }
    free(C->Kedge);
    free(C->beta);
    free(C->gam);
    free(C->gam_next);
}

static void circ_swap_gamma(circ_t *C)
{
    double *t = C->gam;
    C->gam = C->gam_next;
    C->gam_next = t;
}

/* gamma_2 = K^{(1,2)} copied into C->gam. */
static void circ_gamma_first(circ_t *C)
{
    memcpy(C->gam, C->Kedge[0], (size_t)(cn(C, 0) * cn(C, 1)) * sizeof(double));
}

/* Sinkhorn for circle structure, Algorithm 3 (same stopping rule as the tree). */
int orc_circle_sinkhorn_ex(int K, int d, const long *off, const double *pts, const double *closing,
                           const double *mu, double eta, int max_sweeps, double delta, double *phi_cat,
                           double *S_hist, int *sweeps_done)
{
    if (K < 3 || eta <= 0.0 || d < 1) return ORC_EINVAL;
    circ_t C = {K, d, off, pts, eta, NULL, NULL, NULL, NULL, closing};
    int rc = circ_alloc(&C);
    double **phi = (double **)malloc((size_t)K * sizeof(double *));
    double *phi_old = (double *)malloc((size_t)off[K] * sizeof(double));
    long nmax = 0;
    for (int k = 0; k < K; ++k)
        if (cn(&C, k) > nmax) nmax = cn(&C, k);
    double *den = (double *)malloc((size_t)nmax * sizeof(double));
    if (rc != ORC_OK || !phi || !phi_old || !den) {
        circ_free(&C);
        free(phi);
        free(phi_old);
        free(den);
        return ORC_ENOMEM;
    }
    for (int k = 0; k < K; ++k) phi[k] = phi_cat + off[k];

    for (int k = K - 1; k >= 1; --k) circ_beta(&C, (const double *const *)phi, k);

    rc = ORC_MAXITER;
    int r;
    for (r = 0; r < max_sweeps; ++r) {
        memcpy(phi_old, phi_cat, (size_t)off[K] * sizeof(double));
        circ_inner_root(&C, (const double *const *)phi, den);
        for (long i = 0; i < cn(&C, 0); ++i) phi[0][i] = mu[i] / den[i];
        for (int k = 1; k < K; ++k) {
            if (k == 1) {
                circ_gamma_first(&C);
            } else {
                circ_gamma_step(&C, (const double *const *)phi, k);
                circ_swap_gamma(&C);
            }
            circ_inner_beta_gamma(&C, (const double *const *)phi, k, C.gam, den);
            const double *muk = mu + off[k];
            for (long i = 0; i < cn(&C, k); ++i) phi[k][i] = muk[i] / den[i];
        }
        for (int k = K - 1; k >= 1; --k) circ_beta(&C, (const double *const *)phi, k);

        double s1 = 0.0, s2 = 0.0;
        for (long i = 0; i < off[K]; ++i)
            if (mu[i] > 0.0) s1 += mu[i] * log(phi_old[i]);
        for (long i = 0; i < cn(&C, 0); ++i)
            if (mu[i] > 0.0) s2 += (mu[i] / phi[0][i]) * phi_old[i];
        S_hist[r] = eta * (s1 - s2);

        for (long i = 0; i < off[K]; ++i)
            if (!isfinite(phi_cat[i])) {
                rc = ORC_ENUMERIC;
                break;
            }
        if (rc == ORC_ENUMERIC) {
            ++r;
            break;
        }
        if (delta > 0.0 && r >= 1 && fabs(S_hist[r] - S_hist[r - 1]) < delta) {
            rc = ORC_OK;
            ++r;
            break;
        }
    }
    *sweeps_done = r;
    circ_free(&C);
    free(phi);
    free(phi_old);
    free(den);
    return rc;
}

/* Marginals at fixed phi, Theorem 4.3:
 *   P_1 = phi^1 (.) <K^{(1,2)}, (phi^2 (.) alpha^{(2,1)})^T>,
 *   P_k = phi^k (.) <alpha^{(k,1)}, (phi^1 (.) lambda^{(1,k)})^T>. */
int orc_circle_marginals_ex(int K, int d, const long *off, const double *pts, const double *closing,
                            double eta, const double *phi_cat, double *P)
{
    if (K < 3 || eta <= 0.0) return ORC_EINVAL;
    circ_t C = {K, d, off, pts, eta, NULL, NULL, NULL, NULL, closing};
    long nmax = 0;
    for (int k = 0; k < K; ++k)
        if (cn(&C, k) > nmax) nmax = cn(&C, k);
    double *den = (double *)malloc((size_t)nmax * sizeof(double));
    const double **phi = (const double **)malloc((size_t)K * sizeof(double *));
    if (circ_alloc(&C) != ORC_OK || !den || !phi) {
        circ_free(&C);
        free(den);
        free(phi);
        return ORC_ENOMEM;
    }
    for (int k = 0; k < K; ++k) phi[k] = phi_cat + off[k];
    for (int k = K - 1; k >= 1; --k) circ_beta(&C, phi, k);
    circ_inner_root(&C, phi, den);
    for (long i = 0; i < cn(&C, 0); ++i) P[i] = phi[0][i] * den[i];
    for (int k = 1; k < K; ++k) {
        if (k == 1) {
            circ_gamma_first(&C);
        } else {
            circ_gamma_step(&C, phi, k);
            circ_swap_gamma(&C);
        }
        circ_inner_beta_gamma(&C, phi, k, C.gam, den);
        for (long i = 0; i < cn(&C, k); ++i) P[off[k] + i] = phi[k][i] * den[i];
    }
    circ_free(&C);
    free(den);
    free(phi);
    return ORC_OK;
}

int orc_circle_sinkhorn(int K, int d, const long *off, const double *pts, const double *mu,
                        double eta, int max_sweeps, double delta, double *phi_cat,
                        double *S_hist, int *sweeps_done)
{
    return orc_circle_sinkhorn_ex(K, d, off, pts, NULL, mu, eta, max_sweeps, delta, phi_cat, S_hist,
                                  sweeps_done);
}

int orc_circle_marginals(int K, int d, const long *off, const double *pts, double eta,
                         const double *phi_cat, double *P)
{
    return orc_circle_marginals_ex(K, d, off, pts, NULL, eta, phi_cat, P);
}

/* Pair marginal Pi_{1,k} of the circle at fixed phi (Sec. 6.3): the sum of K (.) Phi over
 * every index but i_1 and i_k.  Summing the circle's chain on both sides of the pair,
 *   Pi_{1,k}[i][j] = phi^1_i lambda^{(1,k)}[i][j] alpha^{(k,1)}[j][i] phi^k_j,
 * with lambda^{(1,2)} = K^{(1,2)} (Theorem 4.3's matrices; out is n_1 x n_k row-major,
 * k = 2..K in the paper's numbering, 1..K-1 here). */
int orc_circle_pair_marginal(int K, int d, const long *off, const double *pts, const double *closing,
                             double eta, const double *phi_cat, int k, double *out)
{
    if (K < 3 || eta <= 0.0 || k < 1 || k >= K) return ORC_EINVAL;
    circ_t C = {K, d, off, pts, eta, NULL, NULL, NULL, NULL, closing};
    const double **phi = (const double **)malloc((size_t)K * sizeof(double *));
    if (circ_alloc(&C) != ORC_OK || !phi) {
        circ_free(&C);
        free(phi);
        return ORC_ENOMEM;
    }
    for (int q = 0; q < K; ++q) phi[q] = phi_cat + off[q];
    for (int q = K - 1; q >= 1; --q) circ_beta(&C, phi, q);
    circ_gamma_first(&C);
    for (int q = 2; q <= k; ++q) {
        circ_gamma_step(&C, phi, q);
        circ_swap_gamma(&C);
    }
    const long n1 = cn(&C, 0), nk = cn(&C, k);
    for (long i = 0; i < n1; ++i)
        for (long j = 0; j < nk; ++j)
            out[i * nk + j] = ((phi[0][i] * C.gam[i * nk + j]) * C.beta[k][j * n1 + i]) * phi[k][j];
    circ_free(&C);
    free(phi);
    return ORC_OK;
}

/* Pair marginal of a tree edge {p(k), k} at fixed phi (Theorem 4.1 applied to the pair):
 *   Pi_{p,k}[i][j] = (phi^p gamma_p prod_{t in C_p, t != k} beta_t)_i K^{(p,k)}[i][j]
 *                    (phi^k prod_{t in C_k} beta_t)_j,
 * out is n_p x n_k row-major; edge costs weighted by edge_w (NULL = 1). */
int orc_tree_pair_marginal(int K, int d, const long *off, const double *pts, const int *parent,
                           const double *edge_w, double eta, const double *phi_cat, int k, double *out)
{
    if (tree_check(K, parent) != ORC_OK || eta <= 0.0 || k < 1 || k >= K) return ORC_EINVAL;
    tree_t T = {K, d, off, pts, parent, eta, NULL, NULL, NULL, edge_w, NULL};
    if (tree_alloc(&T) != ORC_OK) {
        tree_free(&T);
        return ORC_ENOMEM;
    }
    const double **phi = (const double **)malloc((size_t)K * sizeof(double *));
    for (int q = 0; q < K; ++q) phi[q] = phi_cat + off[q];
    for (int q = K - 1; q >= 1; --q) compute_beta(&T, phi, q);
    for (int q = 0; q < K; ++q) compute_gamma(&T, phi, q);
    const int p = parent[k];
    const long np_ = tn(&T, p), nk = tn(&T, k);
    double *u = (double *)malloc((size_t)np_ * sizeof(double));
    double *w = (double *)malloc((size_t)nk * sizeof(double));
    double *Kpk = (double *)malloc((size_t)(np_ * nk) * sizeof(double));
    child_product(&T, p, k, u);
    for (long i = 0; i < np_; ++i) u[i] = (phi[p][i] * T.gamma[p][i]) * u[i];
    child_product(&T, k, -1, w);
    for (long j = 0; j < nk; ++j) w[j] = phi[k][j] * w[j];
    kernel_matrix(d, np_, tpts(&T, p), nk, tpts(&T, k), edge_eta(&T, k), Kpk);
    for (long i = 0; i < np_; ++i)
        for (long j = 0; j < nk; ++j) out[i * nk + j] = (u[i] * Kpk[i * nk + j]) * w[j];
    free(u);
    free(w);
    free(Kpk);
    free(phi);
    tree_free(&T);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Point binning (not in the paper; the GPU library's node ordering).
 *   u_c    = x_c * s_c + o_c           (two separately rounded FP64 operations)
 *   cell_c = clamp(floor(u_c), 0, n-1)
 *   tile_c = cell_c / T,  tiles per dim = ceil(n / T)
 *   tile   = row-major linearisation with coordinate 0 slowest
 * perm lists point indices sorted by tile, ties in ascending original index
 * (a stable counting sort); tile_off[t] is the first sorted position of tile
 * t, tile_off[ntiles] = n_pts.  cell is n_pts x d in original order.
 *
 * With 0 <= sub_dim < d the points of one tile are further ordered by their
 * tile-relative cell in dimension sub_dim, r = cell_{sub_dim} mod T, ties again
 * in ascending original index: the sort key is (tile, r, index).  This is the
 * order the 3-D fast-summation path keeps its points in; tile_off is unchanged
 * (a tile's points stay contiguous).  sub_dim < 0 gives the plain tile order. */
int orc_bin_points_sub(int d, long n_pts, const double *x, const double *s, const double *o,
                       int n, int T, int sub_dim, int *cell, int *tile, int *perm, int *tile_off)
{
    if (d < 1 || d > 3 || n < 1 || T < 1 || sub_dim >= d) return ORC_EINVAL;
    int tpd = (n + T - 1) / T;
    long ntiles = 1;
    for (int c = 0; c < d; ++c) ntiles *= tpd;
    for (long i = 0; i < n_pts; ++i) {
        long t = 0;
        for (int c = 0; c < d; ++c) {
            /* volatile: the product is rounded before the add (no FMA). */
            volatile double prod = x[i * d + c] * s[c];
            double u = prod + o[c];
            double f = floor(u);
            int ci;
            if (!(f >= 0.0))
                ci = 0;
            else if (f > (double)(n - 1))
                ci = n - 1;
            else
                ci = (int)f;
            cell[i * d + c] = ci;
            t = t * tpd + ci / T;
        }
        tile[i] = (int)t;
    }
    for (long t = 0; t <= ntiles; ++t) tile_off[t] = 0;
    for (long i = 0; i < n_pts; ++i) tile_off[tile[i] + 1] += 1;
    for (long t = 0; t < ntiles; ++t) tile_off[t + 1] += tile_off[t];
    /* stable counting sort by the bucket (tile, r): ntiles * R buckets, R = T with a
     * sub-key and 1 without; points enter their bucket in ascending index order */
    const long R = sub_dim >= 0 ? T : 1;
    long *bucket_off = (long *)calloc((size_t)(ntiles * R + 1), sizeof(long));
    if (!bucket_off) return ORC_ENOMEM;
    for (long i = 0; i < n_pts; ++i) {
        long b = (long)tile[i] * R + (sub_dim >= 0 ? cell[i * d + sub_dim] % T : 0);
        bucket_off[b + 1] += 1;
    }
    for (long b = 0; b < ntiles * R; ++b) bucket_off[b + 1] += bucket_off[b];
    for (long i = 0; i < n_pts; ++i) {
        long b = (long)tile[i] * R + (sub_dim >= 0 ? cell[i * d + sub_dim] % T : 0);
        perm[bucket_off[b]++] = (int)i;
    }
    free(bucket_off);
    return ORC_OK;
}

int orc_bin_points(int d, long n_pts, const double *x, const double *s, const double *o,
                   int n, int T, int *cell, int *tile, int *perm, int *tile_off)
{
    return orc_bin_points_sub(d, n_pts, x, s, o, n, T, -1, cell, tile, perm, tile_off);
}
