/*
 * prtgs_oracle.c -- plain, slow CPU reference for the PRTGS transfer path.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
 * leg of the benchmark call this code; the HIP library never links, loads or
 * calls it, and the two share no source.  Everything here is double
 * precision and brute force: every traced ray is tested against every other
 * Gaussian, with no acceleration structure, no blocking and no reordering.
 *
 * What it computes (PRTGS, arXiv 2408.03538):
 *   - a stratified set of S directions on the sphere and the real spherical
 *     harmonics Y_k at them (SH projection, Eq. 8-11);
 *   - for each source splat i and direction w with n_i . w > 0, the
 *     transmittance V along the ray x(t) = mu_i + t w through the other 3D
 *     Gaussians (Eq. 1-2), V = prod(1 - alpha_j) as in the alpha blend of
 *     Eq. 4, with alpha_j = o_j exp(-d_j^2 / 2) at the peak density of
 *     Gaussian j along the ray (the reading of Eq. 27 used here);
 *   - the diffuse transfer vector t_i[k] = (4 pi / S) sum_s V c Y_k(w_s),
 *     c = max(0, n_i . w_s)  (Eq. 7, 9, 29; the receiver's rho/pi is left to
 *     the consumer);
 *   - one interreflection bounce (Eq. 20-22, 30-33): the hits of each ray,
 *     taken front to back, weight the direct transfer of the hit splat by
 *     w_j = alpha_j T_j (Eq. 4 / Eq. 26 without the argmax) and its albedo
 *     rho_j / pi.
 * Relighting (Eq. 14) and gradients live in the Python side of the oracle.
 *
 * Cutoffs, shared verbatim with the GPU path (array `cut`):
 *   cut[0] sigma_cut : a Gaussian is hit iff d^2 <= sigma_cut^2
 *   cut[1] t_min     : ... and its peak lies at t* > t_min
 *   cut[2] T_eps     : a transmittance below T_eps counts as 0 (opaque)
 *   cut[3] alpha_min : hits with alpha < alpha_min are ignored
 *   cut[4] alpha_max : alpha is clamped to alpha_max
 *   cut[5] c_min     : a ray is traced iff c = n_i . w > c_min (0 on the GPU
 *                      path; other values only move the hemisphere threshold
 *                      to check the deviation bound of its near-threshold rays)
 *
 * Near-threshold margins (array `mar`), used only to bound how much a result
 * computed in another precision may legitimately differ (both resolutions of
 * a predicate that lies within rounding of its threshold are correct):
 *   mar[0] |c| below which the hemisphere test is ambiguous
 *   mar[1] margin of d^2 against sigma_cut^2, times (1 + kappa_j)
 *   mar[2] margin of t* against t_min: mar[2] (1 + d) / |W w| + mar[4] |t*|
 *   mar[3] relative margin of the transmittance against T_eps (and t_same)
 *   mar[4] the relative part of the t* margin; two peak depths count as tied
 *          when they differ by at most the sum of their t* margins
 * with kappa_j = s_max,j / s_min,j the anisotropy of Gaussian j, d = sqrt(d^2)
 * and |W w| = sqrt(w^T Sigma_j^-1 w).  These are the error scales of an FP32
 * evaluation that forms p = W x from the exact offset x between the ray point
 * and the centre (W = diag(1/s) R^T, Eq. 2) and refines t* by a Newton step:
 * rounding W and W x moves the thin-axis component of p by a few eps times
 * |x| / s_min, and |x| <= 3 s_max for a Gaussian the ray reaches, so d^2
 * moves by O(eps kappa); the step leaves t* off by the error of p along W w
 * over |W w|, O(eps (1 + d) / |W w|).  Neither depends on the distance to
 * the ray origin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state advances by the  */
/* golden-ratio increment and each output is the state passed through the    */
/* variant-13 finaliser.  Output number `index` (0-based) of the stream that  */
/* starts at `seed` therefore depends on seed + (index + 1) * gamma only.    */
/* ------------------------------------------------------------------------ */
uint64_t ora_splitmix64(uint64_t seed, uint64_t index)
{
    uint64_t z = seed + (index + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform double in [0, 1) from the top 53 bits of output `index` */
static double ora_uniform(uint64_t seed, uint64_t index)
{
    return (double)(ora_splitmix64(seed, index) >> 11) * (1.0 / 9007199254740992.0);
}

/* Grid of the stratification: n_u bands in z times n_v sectors in phi, with
 * n_u the largest divisor of S not above floor(sqrt(S)). */
void ora_grid(int S, int* nu, int* nv)
{
    int r = (int)floor(sqrt((double)S));
    while (r * r > S) --r;
    while ((r + 1) * (r + 1) <= S) ++r;
    int u = 1;
    for (int d = 1; d <= r; ++d)
        if (S % d == 0) u = d;
    *nu = u;
    *nv = S / u;
}

/* S equal-area stratified directions.  Stratum s = a * n_v + b covers
 * z in [1 - 2(a+1)/n_u, 1 - 2a/n_u] and phi in [2 pi b/n_v, 2 pi (b+1)/n_v],
 * of area 4 pi / S; one jittered point (xi = U(2s), eta = U(2s+1)) is drawn
 * in it.  The result is rounded to float and promoted back, so that FP32 and
 * FP64 consumers share exactly the same direction. */
void ora_directions(int S, uint64_t seed, double* dirs)
{
    int nu, nv;
    ora_grid(S, &nu, &nv);
    for (int s = 0; s < S; ++s) {
        int a = s / nv, b = s % nv;
        double xi = ora_uniform(seed, 2u * (uint64_t)s);
        double eta = ora_uniform(seed, 2u * (uint64_t)s + 1u);
        double z = 1.0 - 2.0 * ((double)a + xi) / (double)nu;
        double phi = 2.0 * ORA_PI * ((double)b + eta) / (double)nv;
        double r = sqrt(fmax(0.0, 1.0 - z * z));
        dirs[3 * s + 0] = (double)(float)(r * cos(phi));
        dirs[3 * s + 1] = (double)(float)(r * sin(phi));
        dirs[3 * s + 2] = (double)(float)z;
    }
}

/* Associated Legendre function P_l^m(x), Condon-Shortley phase included,
 * by the textbook three-term recurrence in l. */
static double ora_legendre(int l, int m, double x)
{
    double somx2 = sqrt(fmax(0.0, (1.0 - x) * (1.0 + x)));
    double pmm = 1.0;
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * somx2;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

/* Real orthonormal SH, index k = l^2 + l + m (Eq. 8-10):
 *   m > 0: sqrt2 K_l^m P_l^m(cos th) cos(m ph)
 *   m < 0: sqrt2 K_l^|m| P_l^|m|(cos th) sin(|m| ph)
 *   m = 0: K_l^0 P_l(cos th)
 * with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), at the unit vector w/|w|. */
void ora_sh_basis(int L, const double* w, double* Y)
{
    double len = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double x = w[0] / len, y = w[1] / len, z = w[2] / len;
    double ph = atan2(y, x);
    for (int l = 0; l < L; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double ratio = 1.0; /* (l-|m|)! / (l+|m|)! */
            for (int f = l - am + 1; f <= l + am; ++f) ratio /= (double)f;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * ORA_PI) * ratio);
            double P = ora_legendre(l, am, z);
            double v;
            if (m > 0) v = sqrt(2.0) * K * P * cos(am * ph);
            else if (m < 0) v = sqrt(2.0) * K * P * sin(am * ph);
            else v = K * P;
            Y[l * l + l + m] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Gaussians: Sigma = R S S^T R^T (Eq. 2), so Sigma^-1 = R diag(s^-2) R^T.   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double mu[3];
    double sinv[9]; /* row-major Sigma^{-1} */
    double o;
    double smin;    /* smallest and largest scale, for the rounding margins only */
    double smax;
} OraGauss;

static void ora_rotation(const double* q, double* R)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static OraGauss* ora_setup(int n, const double* means, const double* quats,
                           const double* log_scales, const double* opacity)
{
    OraGauss* g = (OraGauss*)malloc(sizeof(OraGauss) * (size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; ++j) {
        double R[9], inv2[3];
        ora_rotation(quats + 4 * (size_t)j, R);
        g[j].smin = INFINITY;
        g[j].smax = 0.0;
        for (int a = 0; a < 3; ++a) {
            double s = exp(log_scales[3 * (size_t)j + a]);
            inv2[a] = 1.0 / (s * s);
            if (s < g[j].smin) g[j].smin = s;
            if (s > g[j].smax) g[j].smax = s;
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int a = 0; a < 3; ++a) acc += R[3 * r + a] * inv2[a] * R[3 * c + a];
                g[j].sinv[3 * r + c] = acc;
            }
        for (int a = 0; a < 3; ++a) g[j].mu[a] = means[3 * (size_t)j + a];
        g[j].o = opacity[j];
    }
    return g;
}

static void matvec3(const double* M, const double* v, double* out)
{
    for (int r = 0; r < 3; ++r) out[r] = M[3 * r] * v[0] + M[3 * r + 1] * v[1] + M[3 * r + 2] * v[2];
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* One ray-Gaussian test.  The ray x(t) = org + t w reaches the peak density
 * of Gaussian g where (x(t) - mu)^T Sigma^-1 (x(t) - mu) is smallest:
 *   t* = w^T Sigma^-1 (mu - org) / (w^T Sigma^-1 w),
 * d^2 is that quadratic form at x(t*), and alpha = o exp(-d^2 / 2) (Eq. 1,
 * Eq. 27 as read here).  Returns 1 on a hit, with ambiguity flags. */
typedef struct {
    double t, alpha;
    double alpha_if_hit; /* alpha it has, or would have were it a hit */
    double mt;           /* margin of t (0 without margins) */
    int j;
    int amb; /* the hit predicate is within its margin */
} OraHit;

/* The t* margin at peak depth t, d^2 and wSw = w^T Sigma^-1 w (mar[2] above). */
static double ora_t_margin(const double* mar, double t, double d2, double wSw)
{
    return mar ? mar[2] * (1.0 + sqrt(fmax(d2, 0.0))) / sqrt(wSw) + mar[4] * fabs(t) : 0.0;
}

static int ora_test(const OraGauss* g, const double* org, const double* w, const double* cut,
                    const double* mar, double* t_out, double* alpha_out, int* amb_out, double* mt_out)
{
    double rel[3] = {g->mu[0] - org[0], g->mu[1] - org[1], g->mu[2] - org[2]};
    double sw[3];
    matvec3(g->sinv, w, sw);
    double t = dot3(rel, sw) / dot3(w, sw);
    double e[3] = {org[0] + t * w[0] - g->mu[0], org[1] + t * w[1] - g->mu[1], org[2] + t * w[2] - g->mu[2]};
    double se[3];
    matvec3(g->sinv, e, se);
    double d2 = dot3(e, se);
    double cut2 = cut[0] * cut[0];
    int hit = (t > cut[1]) && (d2 <= cut2);
    double alpha = 0.0;
    if (hit) {
        alpha = g->o * exp(-0.5 * d2);
        if (alpha > cut[4]) alpha = cut[4];
        if (alpha < cut[3]) hit = 0;
    }
    int amb = 0;
    if (mar) {
        /* FP32 evaluation error of d^2 and t* (see mar[] above) */
        double md2 = mar[1] * (1.0 + g->smax / g->smin);
        double mt = ora_t_margin(mar, t, d2, dot3(w, sw));
        if (fabs(d2 - cut2) <= md2 && t > cut[1] - mt) amb = 1;
        if (fabs(t - cut[1]) <= mt && d2 <= cut2 + md2) amb = 1;
        if (cut[3] > 0.0) {
            double a_raw = fmin(g->o * exp(-0.5 * d2), cut[4]);
            if (fabs(a_raw - cut[3]) <= 1e-5 * cut[3] + 0.5 * a_raw * md2 && t > cut[1] && d2 <= cut2) amb = 1;
        }
    }
    *t_out = t;
    *alpha_out = alpha;
    *amb_out = amb;
    if (mt_out) *mt_out = ora_t_margin(mar, t, d2, dot3(w, sw));
    return hit;
}

/* The alpha Gaussian g would contribute to the ray org + t w were its hit
 * predicate true (used for the deviation bounds of ambiguous misses). */
static double ora_alpha_if_hit(const OraGauss* g, const double* org, const double* w, const double* cut)
{
    double rel[3] = {g->mu[0] - org[0], g->mu[1] - org[1], g->mu[2] - org[2]};
    double sw[3], se[3];
    matvec3(g->sinv, w, sw);
    double tt = dot3(rel, sw) / dot3(w, sw);
    double e[3] = {org[0] + tt * w[0] - g->mu[0], org[1] + tt * w[1] - g->mu[1], org[2] + tt * w[2] - g->mu[2]};
    matvec3(g->sinv, e, se);
    return fmin(g->o * exp(-0.5 * dot3(e, se)), cut[4]);
}

/* Transmittance along one ray through all Gaussians but `self` (Eq. 4's
 * product), with the bounds lo/hi that a different resolution of the
 * ambiguous predicates could give. */
static double ora_ray_vis(const OraGauss* g, int n, int self, const double* w, const double* cut,
                          const double* mar, double* vlo, double* vhi)
{
    const double* org = g[self].mu;
    double v = 1.0, v_def = 1.0, v_amb = 1.0;
    for (int j = 0; j < n; ++j) {
        if (j == self) continue;
        double t, alpha;
        int amb;
        int hit = ora_test(&g[j], org, w, cut, mar, &t, &alpha, &amb, NULL);
        if (hit) v *= 1.0 - alpha;
        if (amb) {
            /* the other resolution: hit with the alpha it would have */
            double d_alpha = hit ? alpha : ora_alpha_if_hit(&g[j], org, w, cut);
            v_amb *= 1.0 - d_alpha;
        } else if (hit) {
            v_def *= 1.0 - alpha;
        }
    }
    double T_eps = cut[2];
    double lo = v_def * v_amb, hi = v_def;
    if (mar) {
        if (lo < T_eps * (1.0 + mar[3])) lo = 0.0;
        if (hi < T_eps * (1.0 - mar[3])) hi = 0.0;
    } else {
        if (lo < T_eps) lo = 0.0;
        if (hi < T_eps) hi = 0.0;
    }
    if (vlo) *vlo = lo;
    if (vhi) *vhi = hi;
    return v < T_eps ? 0.0 : v;
}

static int ora_threads(int requested)
{
#ifdef _OPENMP
    if (requested > 0) return requested;
    return omp_get_max_threads();
#else
    (void)requested;
    return 1;
#endif
}

/* Direct transfer of the listed sources (Eq. 29 without the receiver's BRDF):
 *   t[i][k] = (4 pi / S) sum_s V_is max(0, n_i . w_s) Y_k(w_s).
 * vis[i][s] receives V for traced rays and -1 for rays with n_i . w_s <= 0.
 * allow[i][k] receives the legitimate-deviation bound of each coefficient.
 * vlo/vhi[i][s] (may be NULL) receive the range of V over the other
 * resolutions of the ray's near-threshold predicates (lo = hi = V without
 * any), for rays that are traced or whose hemisphere test is ambiguous, and
 * -1 for the rest. */
int ora_direct(int n, const double* means, const double* quats, const double* log_scales,
               const double* opacity, const double* normals, int S, const double* dirs, int K,
               const double* Y, const double* cut, const double* mar, const int* sources, int count,
               double* t_out, double* vis_out, double* allow_out, double* vlo_out, double* vhi_out, int threads)
{
    OraGauss* g = ora_setup(n, means, quats, log_scales, opacity);
    double wq = 4.0 * ORA_PI / (double)S;
    int nt = ora_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int q = 0; q < count; ++q) {
        int i = sources[q];
        const double* nrm = normals + 3 * (size_t)i;
        double* t = t_out + (size_t)q * K;
        double* al = allow_out ? allow_out + (size_t)q * K : NULL;
        for (int k = 0; k < K; ++k) {
            t[k] = 0.0;
            if (al) al[k] = 0.0;
        }
        for (int s = 0; s < S; ++s) {
            const double* w = dirs + 3 * (size_t)s;
            double c = dot3(nrm, w);
            int amb_c = mar && fabs(c - cut[5]) <= mar[0];
            double vis = -1.0, vlo = -1.0, vhi = -1.0;
            if (c > cut[5] || amb_c) {
                double lo, hi;
                double v = ora_ray_vis(g, n, i, w, cut, mar, &lo, &hi);
                vlo = mar ? fmin(lo, v) : v;
                vhi = mar ? fmax(hi, v) : v;
                if (c > cut[5]) {
                    vis = v;
                    for (int k = 0; k < K; ++k) t[k] += wq * v * c * Y[(size_t)s * K + k];
                }
                if (al) {
                    double dev = (c > cut[5] ? c : 0.0) * (hi - lo);
                    if (amb_c) dev += fabs(c);
                    for (int k = 0; k < K; ++k) al[k] += wq * fabs(Y[(size_t)s * K + k]) * dev;
                }
            }
            if (vis_out) vis_out[(size_t)q * S + s] = vis;
            if (vlo_out) vlo_out[(size_t)q * S + s] = vlo;
            if (vhi_out) vhi_out[(size_t)q * S + s] = vhi;
        }
    }
    free(g);
    return 0;
}

/* Visibility of single rays: V[r] for the ray from the centre of Gaussian
 * sources[r] along the unit direction w[r] (Eq. 4's product over every other
 * Gaussian, 0 below T_eps), for the per-ray gradient references. */
int ora_rays_vis(int n, const double* means, const double* quats, const double* log_scales,
                 const double* opacity, int count, const int* sources, const double* w, const double* cut,
                 double* V, int threads)
{
    OraGauss* g = ora_setup(n, means, quats, log_scales, opacity);
    int nt = ora_threads(threads);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int r = 0; r < count; ++r)
        V[r] = ora_ray_vis(g, n, sources[r], w + 3 * (size_t)r, cut, NULL, NULL, NULL);
    free(g);
    return 0;
}

/* Indices of every Gaussian that some traced ray of the listed sources hits
 * (mark[j] = 1), ambiguous hits included. */
int ora_hit_set(int n, const double* means, const double* quats, const double* log_scales,
                const double* opacity, const double* normals, int S, const double* dirs,
                const double* cut, const double* mar, const int* sources, int count,
                unsigned char* mark, int threads)
{
    OraGauss* g = ora_setup(n, means, quats, log_scales, opacity);
    memset(mark, 0, (size_t)n);
    int nt = ora_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int q = 0; q < count; ++q) {
        int i = sources[q];
        const double* nrm = normals + 3 * (size_t)i;
        for (int s = 0; s < S; ++s) {
            const double* w = dirs + 3 * (size_t)s;
            double c = dot3(nrm, w);
            if (!(c > cut[5] || (mar && fabs(c - cut[5]) <= mar[0]))) continue;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                double t, alpha;
                int amb;
                if (ora_test(&g[j], g[i].mu, w, cut, mar, &t, &alpha, &amb, NULL) || amb) mark[j] = 1;
            }
        }
    }
    free(g);
    return 0;
}

static int ora_hit_cmp(const void* pa, const void* pb)
{
    const OraHit* a = (const OraHit*)pa;
    const OraHit* b = (const OraHit*)pb;
    if (a->t < b->t) return -1;
    if (a->t > b->t) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

/* One-bounce indirect transfer of the listed sources (Eq. 20-22, 30-33 with
 * the depth-ordered alpha blend in place of the argmax of Eq. 26):
 *   t_ind[i][c][:] = (4 pi / S) sum_s max(0, n_i.w_s)
 *                    sum_{hits j in (t*, j) order} alpha_j T_j (rho_jc / pi) t_dir[j][:]
 * where T_j is the transmittance in front of hit j and the walk stops after
 * the first hit that brings the transmittance below T_eps.
 * t_dir[j][K] (and its deviation bound allow_dir, may be NULL) is indexed by
 * Gaussian; slot[j] gives the row of Gaussian j in t_dir (-1 = not supplied,
 * which is an error if that Gaussian is hit: return value 1).
 * allow[i][c][k] bounds legitimate deviation from the result. */
int ora_bounce(int n, const double* means, const double* quats, const double* log_scales,
               const double* opacity, const double* normals, const double* albedo, int S,
               const double* dirs, int K, const double* cut, const double* mar, const int* slot,
               const double* t_dir, const double* allow_dir, const int* sources, int count,
               double* t_out, double* allow_out, int threads)
{
    OraGauss* g = ora_setup(n, means, quats, log_scales, opacity);
    double wq = 4.0 * ORA_PI / (double)S;
    int nt = ora_threads(threads);
    int missing = 0;
#pragma omp parallel num_threads(nt)
    {
        OraHit* hits = (OraHit*)malloc(sizeof(OraHit) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
        for (int q = 0; q < count; ++q) {
            int i = sources[q];
            const double* nrm = normals + 3 * (size_t)i;
            double* out = t_out + (size_t)q * 3 * K;
            double* al = allow_out ? allow_out + (size_t)q * 3 * K : NULL;
            for (int k = 0; k < 3 * K; ++k) {
                out[k] = 0.0;
                if (al) al[k] = 0.0;
            }
            for (int s = 0; s < S; ++s) {
                const double* w = dirs + 3 * (size_t)s;
                double c = dot3(nrm, w);
                int amb_c = mar && fabs(c - cut[5]) <= mar[0];
                if (!(c > cut[5] || amb_c)) continue;
                int nh = 0, amb_ray = 0;
                for (int j = 0; j < n; ++j) {
                    if (j == i) continue;
                    double t, alpha, mt;
                    int amb;
                    int hit = ora_test(&g[j], g[i].mu, w, cut, mar, &t, &alpha, &amb, &mt);
                    if (amb) amb_ray = 1;
                    if (amb && !hit) {
                        /* keep it in the list, marked, with the alpha it would
                         * have: it enters the deviation bound but not the sum */
                        hits[nh].t = t;
                        hits[nh].alpha = -1.0;
                        hits[nh].alpha_if_hit = ora_alpha_if_hit(&g[j], g[i].mu, w, cut);
                        hits[nh].mt = mt;
                        hits[nh].j = j;
                        hits[nh].amb = 1;
                        ++nh;
                    } else if (hit) {
                        hits[nh].t = t;
                        hits[nh].alpha = alpha;
                        hits[nh].alpha_if_hit = alpha;
                        hits[nh].mt = mt;
                        hits[nh].j = j;
                        hits[nh].amb = amb;
                        ++nh;
                    }
                }
                qsort(hits, (size_t)nh, sizeof(OraHit), ora_hit_cmp);
                double T = 1.0;
                double cpos = c > cut[5] ? c : 0.0;
                double bound[3 * 64];
                int K3 = 3 * K;
                for (int k = 0; k < K3 && k < 3 * 64; ++k) bound[k] = 0.0;
                int ended = 0;
                /* Deviation bound of this ray, in units of max |rho t_dir / pi|
                 * over its hits.  The blend C = sum_k alpha_k T_k V_k has
                 * |dC/d alpha_h| <= 2 T_h max|V| (the later weights form a
                 * partition of at most unity), and T_h at most the product over
                 * the unambiguous hits in front of h; so each ambiguous hit adds
                 * 2 alpha_h T_h^def.  Two tied hits a, b swap at a cost of
                 * 2 alpha_a alpha_b T max|V|.  Where the walk stops may move: the
                 * tail beyond is below T_eps exp(sum alpha / (1 - alpha)) over the
                 * ambiguous hits.  Two blends never differ by more than 2. */
                double T_def = 1.0, T_run = 1.0, run_alpha = 0.0, units = 0.0, A = 0.0;
                for (int h = 0; h < nh; ++h) {
                    int j = hits[h].j;
                    int row = slot[j];
                    if (row < 0) {
#pragma omp atomic write
                        missing = 1;
                        continue;
                    }
                    const double* td = t_dir + (size_t)row * K;
                    const double* rho = albedo + 3 * (size_t)j;
                    if (mar) {
                        for (int ch = 0; ch < 3; ++ch)
                            for (int k = 0; k < K; ++k) {
                                double m = rho[ch] / ORA_PI * (fabs(td[k]) + (allow_dir ? allow_dir[(size_t)row * K + k] : 0.0));
                                if (m > bound[ch * K + k]) bound[ch * K + k] = m;
                            }
                        if (!ended) {
                            double aa = hits[h].alpha_if_hit;
                            int tied = h > 0 && fabs(hits[h].t - hits[h - 1].t) <= hits[h].mt + hits[h - 1].mt;
                            if (tied) {
                                amb_ray = 1;
                                units += 2.0 * aa * run_alpha * T_run;
                                run_alpha += aa;
                            } else {
                                T_run = T_def;
                                run_alpha = aa;
                            }
                            if (hits[h].amb) {
                                units += 2.0 * aa * T_def;
                                A += aa / (1.0 - aa);
                            }
                        }
                    }
                    if (ended || hits[h].alpha < 0.0) continue;
                    double a = hits[h].alpha;
                    double wgt = a * T;
                    if (c > cut[5])
                        for (int ch = 0; ch < 3; ++ch)
                            for (int k = 0; k < K; ++k)
                                out[ch * K + k] += wq * cpos * wgt * rho[ch] / ORA_PI * td[k];
                    if (al && allow_dir)
                        for (int ch = 0; ch < 3; ++ch)
                            for (int k = 0; k < K; ++k)
                                al[ch * K + k] += wq * cpos * wgt * rho[ch] / ORA_PI * allow_dir[(size_t)row * K + k];
                    T *= 1.0 - a;
                    if (!hits[h].amb) T_def *= 1.0 - a;
                    if (mar && fabs(T - cut[2]) <= mar[3] * cut[2]) amb_ray = 1;
                    if (T < cut[2]) ended = 1;
                }
                if (al && (amb_ray || amb_c)) {
                    double cc = amb_c ? fmax(cpos, fabs(c) + mar[0]) : cpos;
                    units += 2.0 * (1.0 + mar[3]) * cut[2] * exp(fmin(A, 700.0));
                    if (amb_c) units += 1.0;   /* the ray may not be traced at all */
                    if (units > 2.0) units = 2.0;
                    for (int k = 0; k < K3; ++k) al[k] += wq * cc * units * bound[k];
                }
            }
        }
        free(hits);
    }
    free(g);
    return missing;
}

/* Index matrix of the paper's own bounce (Sec. 4.4: the weight of Eq. 26,
 * the same-surface filter after Eq. 27, the argmax per direction): for each
 * ray of the listed sources with c = n_i . w > 0, the hits are walked in
 * (t*, j) order up to the one that takes the transmittance below T_eps; hit j
 * is a candidate if the transmittance T_j in front of it is <= t_same, and
 * weighs W_j = alpha_j T_j max(-w . n_j, 0).  idx = the candidate of largest
 * W (the nearer one on a tie), or -1 when no candidate has W > 0 or the ray
 * is not traced.
 * With `mar`, amb[q][s] = 1 where FP32 evaluation may pick differently.  A
 * hit whose predicate lies within its margin (or two hits with tied t*) may
 * or may not scale the T of every later hit by (1 - alpha): two candidates'
 * weights then move against each other by at most the alphas of such hits
 * lying between them, delta = 1e-4 + that sum.  The ray is ambiguous if a
 * candidate other than the best lies within 2 delta of the best weight, if a
 * hit whose candidacy is uncertain (its predicate, its T against t_same or
 * its facing factor within the margins) could reach the best, if the walk
 * may stop one hit later (T within its margin of T_eps) while the best weight
 * is below 2 T_eps, or if c itself is within its margin of 0. */
int ora_index(int n, const double* means, const double* quats, const double* log_scales, const double* opacity,
              const double* normals, int S, const double* dirs, const double* cut, double t_same, const double* mar,
              const int* sources, int count, int* idx_out, unsigned char* amb_out, int threads)
{
    OraGauss* g = ora_setup(n, means, quats, log_scales, opacity);
    int nt = ora_threads(threads);
#pragma omp parallel num_threads(nt)
    {
        size_t cap = (size_t)(n > 0 ? n : 1);
        OraHit* hits = (OraHit*)malloc(sizeof(OraHit) * cap);
        double* pa = (double*)malloc(sizeof(double) * (cap + 1));   /* uncertain alpha in front of position h */
        double* cw = (double*)malloc(sizeof(double) * cap);         /* candidate weights by position */
        unsigned char* cu = (unsigned char*)malloc(cap);            /* candidacy uncertain */
#pragma omp for schedule(dynamic, 1)
        for (int q = 0; q < count; ++q) {
            int i = sources[q];
            const double* nrm = normals + 3 * (size_t)i;
            for (int s = 0; s < S; ++s) {
                const double* w = dirs + 3 * (size_t)s;
                double c = dot3(nrm, w);
                int amb = mar && fabs(c - cut[5]) <= mar[0];
                int best = -1;
                if (c > cut[5] || amb) {
                    int nh = 0;
                    for (int j = 0; j < n; ++j) {
                        if (j == i) continue;
                        double t, alpha, mt;
                        int a_j;
                        int hit = ora_test(&g[j], g[i].mu, w, cut, mar, &t, &alpha, &a_j, &mt);
                        if (hit || a_j) {
                            hits[nh].t = t;
                            hits[nh].alpha = hit ? alpha : -1.0;
                            hits[nh].alpha_if_hit = hit ? alpha : ora_alpha_if_hit(&g[j], g[i].mu, w, cut);
                            hits[nh].mt = mt;
                            hits[nh].j = j;
                            hits[nh].amb = a_j;
                            ++nh;
                        }
                    }
                    qsort(hits, (size_t)nh, sizeof(OraHit), ora_hit_cmp);
                    double T = 1.0, bestW = 0.0;
                    int best_pos = -1, in_front = 0, eps_amb = 0, walked = 0;
                    pa[0] = 0.0;
                    for (int h = 0; h < nh; ++h) {
                        walked = h + 1;
                        double da = 0.0;
                        if (mar && hits[h].amb) da += hits[h].alpha_if_hit;
                        if (mar && h > 0 && fabs(hits[h].t - hits[h - 1].t) <= hits[h].mt + hits[h - 1].mt)
                            da += fmax(hits[h].alpha_if_hit, hits[h - 1].alpha_if_hit);
                        pa[h + 1] = pa[h] + da;
                        const double* nj = normals + 3 * (size_t)hits[h].j;
                        const double f = -dot3(w, nj);
                        const double fpos = f > 0.0 ? f : 0.0;
                        cw[h] = 0.0;
                        cu[h] = 0;
                        if (hits[h].alpha < 0.0) {
                            /* not a hit here, but it may be one in FP32 */
                            cw[h] = hits[h].alpha_if_hit * T * fpos;
                            cu[h] = 1;
                            continue;
                        }
                        double a = hits[h].alpha;
                        int unc = hits[h].amb;
                        if (mar && in_front && fabs(T - t_same) <= mar[3] * t_same) unc = 1;
                        if (mar && fabs(f) <= mar[0]) unc = 1;
                        double W = a * T * fpos;
                        if (T <= t_same || unc) cw[h] = W;
                        cu[h] = (unsigned char)unc;
                        if (T <= t_same && W > bestW) {
                            bestW = W;
                            best = hits[h].j;
                            best_pos = h;
                        }
                        T *= 1.0 - a;
                        ++in_front;
                        if (mar && fabs(T - cut[2]) <= mar[3] * cut[2]) eps_amb = 1;
                        if (T < cut[2]) break;
                    }
                    if (mar) {
                        for (int h = 0; h < walked; ++h) {
                            if (h == best_pos && !cu[h]) continue;
                            if (cw[h] <= 0.0) continue;
                            int lo = h < best_pos ? h : best_pos, hi = h < best_pos ? best_pos : h;
                            double delta = 1e-4 + (best_pos >= 0 ? pa[hi + 1] - pa[lo] : pa[h + 1]);
                            if (cw[h] >= (1.0 - 2.0 * delta) * bestW) amb = 1;
                        }
                        if (eps_amb && bestW < 2.0 * cut[2]) amb = 1;
                    }
                    if (!(c > cut[5])) best = -1;
                }
                idx_out[(size_t)q * S + s] = best;
                if (amb_out) amb_out[(size_t)q * S + s] = (unsigned char)(amb != 0);
            }
        }
        free(hits);
        free(pa);
        free(cw);
        free(cu);
    }
    free(g);
    return 0;
}
