/*
 * imask_oracle.c - plain FP64 CPU oracle for the ImaSk hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or constant table with the
 * HIP implementation.
 *
 * Everything is double precision, written straight from the definitions:
 *   - ray-driven Joseph projector R_l on the level-l grid and its literal
 *     scatter transpose (R_l is the CT model discretised on the coarse grid
 *     of level l, Sec. 4.1, eq. (CT_sketches));
 *   - block-average decimation T_l and replication T_l^* (Sec. 4.1), the
 *     projection P_l = T_l^* T_l and the full-resolution compensation
 *     S_r = p_r^{-1}(I - sum_l p_l P_l) (Sec. 4.1);
 *   - the sketched operators K_l and their transposes (eq. (CT_sketches));
 *   - the counter-based SplitMix64 draw of the sketch index (Alg. 1: each
 *     iteration picks level i with probability p_i);
 *   - Algorithm 1 (ImaSk) with the Tikhonov prox, a smoothed-TV prox
 *     evaluated by FISTA, and the paper's TV + nonnegativity prox by the
 *     fast gradient projection on the dual (Sec. 4.2 and 4.5);
 *   - the ImaSk-Seq variant of Sec. 5 (dual step first, primal step with the
 *     new dual iterate, extrapolated primal point);
 *   - Alg. 1 with the compact dual tables of Remark 1 (iterates instead of
 *     their projections, plus a running table average);
 *   - Alg. 1 with independent primal and dual sketch draws (Sec. 6 outlook).
 *
 * Conventions: domain [-E,E]^2 (E = extent); level l has N_l = N >> l pixels
 * per side and pixel size h_l = 2E/N_l; pixel (i,j) has centre (x_j, y_i)
 * with x_j = -E + (j+1/2) h_l; rows are y, columns are x, storage row-major.
 * Angle a is theta_a = a*pi/n_angles, or the a-th entry of a given list; bin
 * b has centre s_b = (b - (n_det-1)/2) ds + s0 and the ray is
 * x cos + y sin = s.  Default angles step along rows iff 4a <= n_angles or
 * 4a >= 3 n_angles, listed ones iff |cos| >= |sin|; else along columns.
 * With a source distance D > 0 the rays are those of a fan beam with a flat
 * detector (orc_ray); every other step is the same.
 * Interpolation reads zero outside the image.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_MAX_LEVELS 16

enum { ORC_MODE_PAPER = 0, ORC_MODE_UNBIASED = 1 };
enum { ORC_REG_TIKHONOV = 0, ORC_REG_SMOOTH_TV = 1, ORC_REG_TV = 2 };

/* Angle a: the given list (radians), or a*pi/na.  Row stepping: with the
 * default angles the integer rule 4a <= na or 4a >= 3na (45 and 135 degrees
 * step along rows); with a given list |cos| >= |sin| in FP64. */
static double orc_theta(int a, int na, const double* ang) { return ang ? ang[a] : a * M_PI / na; }

static int orc_rows(int a, int na, const double* ang)
{
    if (ang) return fabs(cos(ang[a])) >= fabs(sin(ang[a]));
    return 4 * a <= na || 4 * a >= 3 * na;
}

/* The line of ray (a, b) as x*ct + y*st = sb, and its stepping axis.
 *
 * Parallel beam (D <= 0): ct = cos(theta_a), st = sin(theta_a), sb the bin
 * centre, as in the conventions above.
 *
 * Fan beam (D > 0, the divergent-beam geometry the paper's operator extends
 * to, Sec. 4.1 and the outlook of Sec. 6): view a puts the source at
 * D (cos beta, sin beta), beta = 2 pi a / na or the a-th listed value, and a
 * flat detector through -Dd (cos beta, sin beta), perpendicular to the
 * central ray; bin b sits at t_b = (b - (nd-1)/2) ds + s0 along
 * (-sin beta, cos beta).  The ray joins the source to that point; (ct, st)
 * is its unit normal and sb = (ct, st) . source.  It steps along rows iff
 * |ct| >= |st| in FP64. */
static void orc_ray(int a, int b, int na, int nd, double ds, double s0, const double* ang, double D, double Dd,
                    double* ct, double* st, double* sb, int* rows)
{
    const double t = (b - (nd - 1) / 2.0) * ds + s0;
    if (!(D > 0.0)) {
        const double th = orc_theta(a, na, ang);
        *ct = cos(th);
        *st = sin(th);
        *sb = t;
        *rows = orc_rows(a, na, ang);
        return;
    }
    const double beta = ang ? ang[a] : 2.0 * M_PI * a / na;
    const double ec[2] = {cos(beta), sin(beta)}, et[2] = {-sin(beta), cos(beta)};
    const double src[2] = {D * ec[0], D * ec[1]};
    const double det[2] = {-Dd * ec[0] + t * et[0], -Dd * ec[1] + t * et[1]};
    const double dir[2] = {det[0] - src[0], det[1] - src[1]};
    const double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1]);
    *ct = -dir[1] / len;
    *st = dir[0] / len;
    *sb = *ct * src[0] + *st * src[1];
    *rows = fabs(*ct) >= fabs(*st);
}

static double orc_pix(const double* z, int nl, long i, long j)
{
    if (i < 0 || j < 0 || i >= nl || j >= nl) return 0.0;
    return z[i * nl + j];
}

/* ---------------------------------------------------------------- Joseph R_l */

/* sino[a][b] = (h_l/|cos|) sum_i interp_j(z[i][.], u)   (row stepping)
 *            = (h_l/|sin|) sum_j interp_i(z[.][j], v)   (column stepping) */
void orc_project(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd, int lvl,
                 const double* z, double* sino)
{
    const int nl = n >> lvl;
    const double hl = 2.0 * E / nl;
    const double c0 = -E + 0.5 * hl; /* centre of pixel 0 along either axis */
#pragma omp parallel for schedule(static)
    for (long ab = 0; ab < (long)na * nd; ++ab) {
        const int a = (int)(ab / nd), b = (int)(ab % nd);
        double ct, st, sb;
        int rows;
        orc_ray(a, b, na, nd, ds, s0, ang, D, Dd, &ct, &st, &sb, &rows);
        double acc = 0.0;
        if (rows) {
            for (int i = 0; i < nl; ++i) {
                const double yi = -E + (i + 0.5) * hl;
                const double u = ((sb - yi * st) / ct - c0) / hl;
                const double fl = floor(u);
                const long j0 = (long)fl;
                const double w = u - fl;
                acc += (1.0 - w) * orc_pix(z, nl, i, j0) + w * orc_pix(z, nl, i, j0 + 1);
            }
            sino[ab] = acc * (hl / fabs(ct));
        } else {
            for (int j = 0; j < nl; ++j) {
                const double xj = -E + (j + 0.5) * hl;
                const double v = ((sb - xj * ct) / st - c0) / hl;
                const double fl = floor(v);
                const long i0 = (long)fl;
                const double w = v - fl;
                acc += (1.0 - w) * orc_pix(z, nl, i0, j) + w * orc_pix(z, nl, i0 + 1, j);
            }
            sino[ab] = acc * (hl / fabs(st));
        }
    }
}

/* The literal transpose of orc_project: the same loops, scattering
 * t*(1-w) and t*w into the two pixels each sample reads. */
void orc_backproject(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd, int lvl,
                     const double* sino, double* z)
{
    const int nl = n >> lvl;
    const double hl = 2.0 * E / nl;
    const double c0 = -E + 0.5 * hl;
    const long dl = (long)nl * nl;
    memset(z, 0, sizeof(double) * dl);
    /* per-thread partial images, summed in thread order afterwards so that
     * the result is reproducible for a fixed thread count */
    const int nt = omp_get_max_threads();
    double* part = (double*)calloc((size_t)nt * dl, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        double* acc = part + (size_t)omp_get_thread_num() * dl;
#pragma omp for schedule(static)
        for (int a = 0; a < na; ++a) {
            for (int b = 0; b < nd; ++b) {
                double ct, st, sb;
                int rows;
                orc_ray(a, b, na, nd, ds, s0, ang, D, Dd, &ct, &st, &sb, &rows);
                const double t = (rows ? hl / fabs(ct) : hl / fabs(st)) * sino[(long)a * nd + b];
                for (int k = 0; k < nl; ++k) {
                    const double ck = -E + (k + 0.5) * hl;
                    const double u = rows ? ((sb - ck * st) / ct - c0) / hl : ((sb - ck * ct) / st - c0) / hl;
                    const double fl = floor(u);
                    const long q0 = (long)fl;
                    const double w = u - fl;
                    if (rows) {
                        if (q0 >= 0 && q0 < nl) acc[(long)k * nl + q0] += t * (1.0 - w);
                        if (q0 + 1 >= 0 && q0 + 1 < nl) acc[(long)k * nl + q0 + 1] += t * w;
                    } else {
                        if (q0 >= 0 && q0 < nl) acc[q0 * nl + k] += t * (1.0 - w);
                        if (q0 + 1 >= 0 && q0 + 1 < nl) acc[(q0 + 1) * nl + k] += t * w;
                    }
                }
            }
        }
    }
    for (int q = 0; q < nt; ++q)
        for (long e = 0; e < dl; ++e) z[e] += part[(size_t)q * dl + e];
    free(part);
}

/* Number of (ray, step) samples with at least one interpolation tap inside
 * the image: the nonzero-sample count of R_l (work accounting only). */
long long orc_count_samples(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd, int lvl)
{
    const int nl = n >> lvl;
    const double hl = 2.0 * E / nl;
    const double c0 = -E + 0.5 * hl;
    long long total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (long ab = 0; ab < (long)na * nd; ++ab) {
        const int a = (int)(ab / nd), b = (int)(ab % nd);
        double ct, st, sb;
        int rows;
        orc_ray(a, b, na, nd, ds, s0, ang, D, Dd, &ct, &st, &sb, &rows);
        for (int k = 0; k < nl; ++k) {
            const double ck = -E + (k + 0.5) * hl;
            const double u = rows ? ((sb - ck * st) / ct - c0) / hl : ((sb - ck * ct) / st - c0) / hl;
            const long q0 = (long)floor(u);
            if (q0 >= -1 && q0 < nl) ++total;
        }
    }
    return total;
}

/* ------------------------------------------------------------ resampling */

/* T_l: 2^l x 2^l block mean (Sec. 4.1). */
void orc_restrict(int n, int lvl, const double* x, double* z)
{
    const int nl = n >> lvl, f = 1 << lvl;
    for (int I = 0; I < nl; ++I)
        for (int J = 0; J < nl; ++J) {
            double s = 0.0;
            for (int a = 0; a < f; ++a)
                for (int b = 0; b < f; ++b) s += x[(long)(I * f + a) * n + (J * f + b)];
            z[(long)I * nl + J] = s / ((double)f * f);
        }
}

/* T_l^*: replication, x[i][j] = z[i >> l][j >> l] (Sec. 4.1). */
void orc_prolong(int n, int lvl, const double* z, double* x)
{
    const int nl = n >> lvl;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) x[(long)i * n + j] = z[(long)(i >> lvl) * nl + (j >> lvl)];
}

/* S_r x = p_0^{-1} (x - sum_{k>0} p_k P_k x) with P_k = T_k^* T_k. */
void orc_compensate(int n, int r, const int* log2f, const double* p, const double* x, double* out)
{
    const long d = (long)n * n;
    double* z = (double*)malloc(sizeof(double) * d);
    double* px = (double*)malloc(sizeof(double) * d);
    for (long q = 0; q < d; ++q) out[q] = x[q];
    for (int k = 1; k < r; ++k) {
        orc_restrict(n, log2f[k], x, z);
        orc_prolong(n, log2f[k], z, px);
        for (long q = 0; q < d; ++q) out[q] -= p[k] * px[q];
    }
    for (long q = 0; q < d; ++q) out[q] /= p[0];
    free(z);
    free(px);
}

/* ------------------------------------------------------ sketched operators */

/* g = K_k x (sinogram), for sketch k of the level set (log2f[0] == 0). */
void orc_sketch_fwd(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd, int r, const int* log2f,
                    const double* p, int mode, int k, const double* x, double* g)
{
    const long d = (long)n * n, m = (long)na * nd;
    double* z = (double*)malloc(sizeof(double) * d);
    if (k > 0) {
        orc_restrict(n, log2f[k], x, z);
        orc_project(n, na, nd, ds, s0, E, ang, D, Dd, log2f[k], z, g);
    } else if (mode == ORC_MODE_PAPER) {
        orc_compensate(n, r, log2f, p, x, z);
        orc_project(n, na, nd, ds, s0, E, ang, D, Dd, 0, z, g);
    } else {
        double* t = (double*)malloc(sizeof(double) * m);
        orc_project(n, na, nd, ds, s0, E, ang, D, Dd, 0, x, g);
        for (int q = 1; q < r; ++q) {
            orc_restrict(n, log2f[q], x, z);
            orc_project(n, na, nd, ds, s0, E, ang, D, Dd, log2f[q], z, t);
            for (long e = 0; e < m; ++e) g[e] -= p[q] * t[e];
        }
        for (long e = 0; e < m; ++e) g[e] /= p[0];
        free(t);
    }
    free(z);
}

/* g = K_k^T y (image), the exact transpose of orc_sketch_fwd. */
void orc_sketch_adj(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd, int r, const int* log2f,
                    const double* p, int mode, int k, const double* y, double* g)
{
    const long d = (long)n * n;
    double* c = (double*)malloc(sizeof(double) * d);
    double* t = (double*)malloc(sizeof(double) * d);
    if (k > 0) {
        const int l = log2f[k];
        const double s = 1.0 / (double)(1L << (2 * l)); /* T_l^T = 4^{-l} T_l^* */
        orc_backproject(n, na, nd, ds, s0, E, ang, D, Dd, l, y, c);
        orc_prolong(n, l, c, g);
        for (long q = 0; q < d; ++q) g[q] *= s;
    } else if (mode == ORC_MODE_PAPER) {
        orc_backproject(n, na, nd, ds, s0, E, ang, D, Dd, 0, y, c);
        orc_compensate(n, r, log2f, p, c, g); /* S_r is symmetric */
    } else {
        orc_backproject(n, na, nd, ds, s0, E, ang, D, Dd, 0, y, g);
        for (int q = 1; q < r; ++q) {
            const int l = log2f[q];
            const double s = 1.0 / (double)(1L << (2 * l));
            orc_backproject(n, na, nd, ds, s0, E, ang, D, Dd, l, y, c);
            orc_prolong(n, l, c, t);
            for (long e = 0; e < d; ++e) g[e] -= p[q] * s * t[e];
        }
        for (long e = 0; e < d; ++e) g[e] /= p[0];
    }
    free(c);
    free(t);
}

/* ---------------------------------------------------------------- draws */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter form: the k-th
 * output (k = 0, 1, ...) of the generator whose state starts at `seed`. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Cumulative thresholds T_j = min(2^32, floor(2^32 * sum_{t<=j} p_t)),
 * with the last one forced to 2^32. */
void orc_thresholds(int r, const double* p, uint64_t* thr)
{
    double cum = 0.0;
    for (int j = 0; j < r; ++j) {
        cum += p[j];
        double t = floor(4294967296.0 * cum);
        if (t > 4294967296.0) t = 4294967296.0;
        thr[j] = (uint64_t)t;
    }
    thr[r - 1] = 4294967296ULL;
}

/* i_k for k = k0 .. k0+count-1 of stream `stream` under base seed `seed`. */
void orc_draws(uint64_t seed, uint32_t stream, uint64_t k0, int count, int r,
               const double* p, int32_t* out)
{
    uint64_t thr[ORC_MAX_LEVELS];
    orc_thresholds(r, p, thr);
    const uint64_t ss = orc_splitmix64(seed, stream);
    for (int q = 0; q < count; ++q) {
        const uint64_t u = orc_splitmix64(ss, k0 + (uint64_t)q) >> 32;
        int j = 0;
        while (u >= thr[j]) ++j;
        out[q] = j;
    }
}

/* ------------------------------------------------------------ smoothed TV */

/* Forward differences with a zero difference at the last row / column. */
static void orc_grad(int n, const double* u, double* g1, double* g2)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const long q = (long)i * n + j;
            g1[q] = (i < n - 1) ? u[q + n] - u[q] : 0.0;
            g2[q] = (j < n - 1) ? u[q + 1] - u[q] : 0.0;
        }
}

/* Adjoint of orc_grad. */
static void orc_grad_adj(int n, const double* q1, const double* q2, double* out)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const long q = (long)i * n + j;
            double s = 0.0;
            if (i >= 1) s += q1[q - n];
            if (i < n - 1) s -= q1[q];
            if (j >= 1) s += q2[q - 1];
            if (j < n - 1) s -= q2[q];
            out[q] = s;
        }
}

/* TV_eps(u) = sum sqrt(|grad u|^2 + eps^2). */
double orc_tv_value(int n, const double* u, double eps)
{
    const long d = (long)n * n;
    double* g1 = (double*)malloc(sizeof(double) * d);
    double* g2 = (double*)malloc(sizeof(double) * d);
    orc_grad(n, u, g1, g2);
    double s = 0.0;
    for (long q = 0; q < d; ++q) s += sqrt(g1[q] * g1[q] + g2[q] * g2[q] + eps * eps);
    free(g1);
    free(g2);
    return s;
}

/* Gradient of TV_eps: grad^T (grad u / sqrt(|grad u|^2 + eps^2)). */
void orc_tv_gradient(int n, const double* u, double eps, double* out)
{
    const long d = (long)n * n;
    double* g1 = (double*)malloc(sizeof(double) * d);
    double* g2 = (double*)malloc(sizeof(double) * d);
    orc_grad(n, u, g1, g2);
    for (long q = 0; q < d; ++q) {
        const double nrm = sqrt(g1[q] * g1[q] + g2[q] * g2[q] + eps * eps);
        g1[q] /= nrm;
        g2[q] /= nrm;
    }
    orc_grad_adj(n, g1, g2, out);
    free(g1);
    free(g2);
}

/* prox of tau*R with R = w TV_eps + (lam/2)|.|^2, approximated by J FISTA
 * iterations (Beck-Teboulle) on h(u) = 1/2|u-v|^2 + tau w TV_eps(u) +
 * tau lam/2 |u|^2, started at u0, step 1/L with L = 1 + tau lam + 8 tau w/eps. */
void orc_tv_prox(int n, const double* v, const double* u0, double tau, double lam,
                 double w, double eps, int J, double* out)
{
    const long d = (long)n * n;
    const double L = 1.0 + tau * lam + 8.0 * tau * w / eps;
    double* uk = (double*)malloc(sizeof(double) * d);
    double* yk = (double*)malloc(sizeof(double) * d);
    double* gr = (double*)malloc(sizeof(double) * d);
    double* un = (double*)malloc(sizeof(double) * d);
    memcpy(uk, u0, sizeof(double) * d);
    memcpy(yk, u0, sizeof(double) * d);
    double t = 1.0;
    for (int it = 0; it < J; ++it) {
        orc_tv_gradient(n, yk, eps, gr);
        for (long q = 0; q < d; ++q) {
            const double gh = (yk[q] - v[q]) + tau * w * gr[q] + tau * lam * yk[q];
            un[q] = yk[q] - gh / L;
        }
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        const double beta = (t - 1.0) / tn;
        for (long q = 0; q < d; ++q) {
            yk[q] = un[q] + beta * (un[q] - uk[q]);
            uk[q] = un[q];
        }
        t = tn;
    }
    memcpy(out, uk, sizeof(double) * d);
    free(uk);
    free(yk);
    free(gr);
    free(un);
}

/* Prox of the paper's TV prior with nonnegativity (Sec. 4.5):
 * argmin_u 1/2|u - b|^2 + gamma TV(u) + chi_{>=0}(u), TV(u) = sum |grad u|_2,
 * by J iterations of the fast gradient projection on the dual (Beck and
 * Teboulle, constrained TV denoising): the dual pair (p1, p2), one vector per
 * pixel in the unit disc, gives u(p) = max(0, b - gamma grad^T p); a step
 * of length 1/(8 gamma) along grad u(p) is projected back onto the discs,
 * with FISTA extrapolation.  (p1, p2) is the warm start on entry and the
 * last iterate on exit (the outer iteration keeps it); u = u(p_J). */
void orc_tv_fgp(int n, const double* b, double gamma, int J, double* p1, double* p2, double* u)
{
    const long d = (long)n * n;
    double* r1 = (double*)malloc(sizeof(double) * d);
    double* r2 = (double*)malloc(sizeof(double) * d);
    double* g1 = (double*)malloc(sizeof(double) * d);
    double* g2 = (double*)malloc(sizeof(double) * d);
    double* w = (double*)malloc(sizeof(double) * d);
    memcpy(r1, p1, sizeof(double) * d);
    memcpy(r2, p2, sizeof(double) * d);
    double t = 1.0;
    for (int it = 0; it < J; ++it) {
        /* u at the extrapolated dual point */
        orc_grad_adj(n, r1, r2, w);
        for (long q = 0; q < d; ++q) w[q] = fmax(0.0, b[q] - gamma * w[q]);
        /* projected gradient step on the dual */
        orc_grad(n, w, g1, g2);
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        const double beta = (t - 1.0) / tn;
        for (long q = 0; q < d; ++q) {
            const double a1 = r1[q] + g1[q] / (8.0 * gamma);
            const double a2 = r2[q] + g2[q] / (8.0 * gamma);
            const double nrm = fmax(1.0, sqrt(a1 * a1 + a2 * a2));
            const double n1 = a1 / nrm, n2 = a2 / nrm;
            r1[q] = n1 + beta * (n1 - p1[q]);
            r2[q] = n2 + beta * (n2 - p2[q]);
            p1[q] = n1;
            p2[q] = n2;
        }
        t = tn;
    }
    orc_grad_adj(n, p1, p2, w);
    for (long q = 0; q < d; ++q) u[q] = fmax(0.0, b[q] - gamma * w[q]);
    free(r1);
    free(r2);
    free(g1);
    free(g2);
    free(w);
}

/* prox_{tau R}(v) for the three regularisers, x^k the current iterate (the
 * smoothed-TV FISTA starts there), tvd the TV dual pair (2 n^2, ORC_REG_TV). */
static void orc_prox(int n, int reg_kind, double tau, double lam, double tv_w, double tv_eps, int tv_inner,
                     const double* v, const double* xk, double* tvd, double* out)
{
    const long d = (long)n * n;
    if (reg_kind == ORC_REG_TIKHONOV) {
        for (long q = 0; q < d; ++q) out[q] = v[q] / (1.0 + tau * lam);
    } else if (reg_kind == ORC_REG_SMOOTH_TV) {
        orc_tv_prox(n, v, xk, tau, lam, tv_w, tv_eps, tv_inner, out);
    } else {
        /* R = w TV + chi_{>=0} + lam/2 |.|^2: the quadratic folds into a
         * rescaled TV denoising problem at v / (1 + tau lam) */
        const double s = 1.0 + tau * lam;
        double* bt = (double*)malloc(sizeof(double) * d);
        for (long q = 0; q < d; ++q) bt[q] = v[q] / s;
        orc_tv_fgp(n, bt, tau * tv_w / s, tv_inner, tvd, tvd + d, out);
        free(bt);
    }
}

/* ------------------------------------------------------------ Algorithm 1 */

/* Runs n_iter iterations of ImaSk (Alg. 1) from the state (x, y, phi, psi)
 * given at iteration k0, in place.  phi holds r full-resolution images
 * (phi_k = K_k^T y at the last refresh), psi holds r sinograms
 * (psi_k = K_k x at the last refresh).  mu = lam.  draws_out[q] receives
 * i_{k0+q}; *epochs accumulates sum_q 2^{-log2f[i_q]} (PAPER cost model) or,
 * in UNBIASED mode, 1 + sum_{k>0} 2^{-log2f[k]} for a full-resolution step. */
int orc_imask_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                  int r, const int* log2f, const double* p, int mode,
                  int reg_kind, double lam, double tv_w, double tv_eps, int tv_inner,
                  double sigma, uint64_t seed, uint32_t stream, uint64_t k0,
                  const double* bdata, int n_iter,
                  double* x, double* y, double* phi, double* psi, double* tvd,
                  int32_t* draws_out, double* epochs)
{
    if (r < 1 || r > ORC_MAX_LEVELS || log2f[0] != 0) return -1;
    const long d = (long)n * n, m = (long)na * nd;
    const double tau = sigma / lam;
    double* gx = (double*)malloc(sizeof(double) * d);
    double* gy = (double*)malloc(sizeof(double) * m);
    double* xi = (double*)malloc(sizeof(double) * d);
    double* zeta = (double*)malloc(sizeof(double) * m);
    double* xn = (double*)malloc(sizeof(double) * d);
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (n_iter > 0 ? n_iter : 1));
    orc_draws(seed, stream, k0, n_iter, r, p, idx);
    double unbiased_full = 1.0;
    for (int k = 1; k < r; ++k) unbiased_full += ldexp(1.0, -log2f[k]);
    for (int it = 0; it < n_iter; ++it) {
        const int k = idx[it];
        /* both refreshed gradients from the old iterates x^k, y^k */
        orc_sketch_adj(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, y, gx);
        orc_sketch_fwd(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, x, gy);
        /* SAGA estimates with the old tables */
        for (long q = 0; q < d; ++q) {
            double avg = 0.0;
            for (int j = 0; j < r; ++j) avg += p[j] * phi[(long)j * d + q];
            xi[q] = gx[q] - phi[(long)k * d + q] + avg;
        }
        for (long e = 0; e < m; ++e) {
            double avg = 0.0;
            for (int j = 0; j < r; ++j) avg += p[j] * psi[(long)j * m + e];
            zeta[e] = gy[e] - psi[(long)k * m + e] + avg;
        }
        /* primal: prox_{tau R}(x - tau xi) */
        {
            double* v = (double*)malloc(sizeof(double) * d);
            for (long q = 0; q < d; ++q) v[q] = x[q] - tau * xi[q];
            orc_prox(n, reg_kind, tau, lam, tv_w, tv_eps, tv_inner, v, x, tvd, xn);
            free(v);
        }
        /* dual: (y + sigma zeta - sigma b)/(1 + sigma) */
        for (long e = 0; e < m; ++e) y[e] = (y[e] + sigma * zeta[e] - sigma * bdata[e]) / (1.0 + sigma);
        memcpy(x, xn, sizeof(double) * d);
        memcpy(phi + (long)k * d, gx, sizeof(double) * d);
        memcpy(psi + (long)k * m, gy, sizeof(double) * m);
        if (draws_out) draws_out[it] = k;
        if (epochs) {
            if (k == 0 && mode == ORC_MODE_UNBIASED) *epochs += unbiased_full;
            else *epochs += ldexp(1.0, -log2f[k]);
        }
    }
    free(gx);
    free(gy);
    free(xi);
    free(zeta);
    free(xn);
    free(idx);
    return 0;
}

/* ImaSk-Seq (Sec. 5, algorithm "Variant ImaSk-Seq"): n_iter iterations from
 * the state (x, xbar, y, phi, psi); mu = lam.  Each iteration, in the order
 * the variant states it:
 *   sample i; psi_new = K_i xbar;
 *   zeta = psi_new - psi_i + sum_j p_j psi_j            (old tables)
 *   y <- (y + sigma zeta - sigma b) / (1 + sigma);
 *   phi_new = K_i^T y                                    (the new y)
 *   xi = phi_new - phi_i + sum_j p_j phi_j               (old tables)
 *   x_new = prox_{tau R}(x - tau xi), tau = sigma / mu;
 *   xbar <- x_new + theta (x_new - x);  x <- x_new;  psi_i, phi_i refreshed.
 * Draws and epoch accounting as in orc_imask_run. */
int orc_imask_seq_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                      int r, const int* log2f, const double* p, int mode,
                      int reg_kind, double lam, double tv_w, double tv_eps, int tv_inner,
                      double sigma, double theta, uint64_t seed, uint32_t stream, uint64_t k0,
                      const double* bdata, int n_iter,
                      double* x, double* xbar, double* y, double* phi, double* psi, double* tvd,
                      int32_t* draws_out, double* epochs)
{
    if (r < 1 || r > ORC_MAX_LEVELS || log2f[0] != 0) return -1;
    const long d = (long)n * n, m = (long)na * nd;
    const double tau = sigma / lam;
    double* gx = (double*)malloc(sizeof(double) * d);
    double* gy = (double*)malloc(sizeof(double) * m);
    double* xn = (double*)malloc(sizeof(double) * d);
    double* v = (double*)malloc(sizeof(double) * d);
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (n_iter > 0 ? n_iter : 1));
    orc_draws(seed, stream, k0, n_iter, r, p, idx);
    double unbiased_full = 1.0;
    for (int k = 1; k < r; ++k) unbiased_full += ldexp(1.0, -log2f[k]);
    for (int it = 0; it < n_iter; ++it) {
        const int k = idx[it];
        /* dual step from the extrapolated point */
        orc_sketch_fwd(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, xbar, gy);
        for (long e = 0; e < m; ++e) {
            double avg = 0.0;
            for (int j = 0; j < r; ++j) avg += p[j] * psi[(long)j * m + e];
            const double zeta = gy[e] - psi[(long)k * m + e] + avg;
            y[e] = (y[e] + sigma * zeta - sigma * bdata[e]) / (1.0 + sigma);
        }
        /* primal step with the new dual iterate */
        orc_sketch_adj(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, y, gx);
        for (long q = 0; q < d; ++q) {
            double avg = 0.0;
            for (int j = 0; j < r; ++j) avg += p[j] * phi[(long)j * d + q];
            const double xi = gx[q] - phi[(long)k * d + q] + avg;
            v[q] = x[q] - tau * xi;
        }
        orc_prox(n, reg_kind, tau, lam, tv_w, tv_eps, tv_inner, v, x, tvd, xn);
        /* extrapolation, then the new iterate and the table refresh */
        for (long q = 0; q < d; ++q) {
            xbar[q] = xn[q] + theta * (xn[q] - x[q]);
            x[q] = xn[q];
        }
        memcpy(phi + (long)k * d, gx, sizeof(double) * d);
        memcpy(psi + (long)k * m, gy, sizeof(double) * m);
        if (draws_out) draws_out[it] = k;
        if (epochs) {
            if (k == 0 && mode == ORC_MODE_UNBIASED) *epochs += unbiased_full;
            else *epochs += ldexp(1.0, -log2f[k]);
        }
    }
    free(gx);
    free(gy);
    free(xn);
    free(v);
    free(idx);
    return 0;
}

/* Alg. 1 with the compact dual tables of Remark 1 (appendix, after the
 * saddle-point SAGA algorithm): instead of psi_i = K_i x^{k_i} the state
 * keeps the iterate itself, z_i = x^{k_i} (r * n^2), and the running average
 * psibar = sum_i p_i psi_i (m).  With linearity one forward projection per
 * step still suffices: d = K_i (x^k - z_i) = psi_new - psi_i, so
 * zeta = d + psibar, psibar <- psibar + p_i d and z_i <- x^k.  Everything
 * else is orc_imask_run. */
int orc_imask_compact_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                          int r, const int* log2f, const double* p, int mode,
                          int reg_kind, double lam, double tv_w, double tv_eps, int tv_inner,
                          double sigma, uint64_t seed, uint32_t stream, uint64_t k0,
                          const double* bdata, int n_iter,
                          double* x, double* y, double* phi, double* zsnap, double* psibar, double* tvd,
                          int32_t* draws_out, double* epochs)
{
    if (r < 1 || r > ORC_MAX_LEVELS || log2f[0] != 0) return -1;
    const long d = (long)n * n, m = (long)na * nd;
    const double tau = sigma / lam;
    double* gx = (double*)malloc(sizeof(double) * d);
    double* dd = (double*)malloc(sizeof(double) * m);
    double* diff = (double*)malloc(sizeof(double) * d);
    double* xi = (double*)malloc(sizeof(double) * d);
    double* xn = (double*)malloc(sizeof(double) * d);
    double* v = (double*)malloc(sizeof(double) * d);
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (n_iter > 0 ? n_iter : 1));
    orc_draws(seed, stream, k0, n_iter, r, p, idx);
    double unbiased_full = 1.0;
    for (int k = 1; k < r; ++k) unbiased_full += ldexp(1.0, -log2f[k]);
    for (int it = 0; it < n_iter; ++it) {
        const int k = idx[it];
        /* both refreshed gradients from the old iterates x^k, y^k */
        orc_sketch_adj(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, y, gx);
        for (long q = 0; q < d; ++q) diff[q] = x[q] - zsnap[(long)k * d + q];
        orc_sketch_fwd(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, diff, dd);
        for (long q = 0; q < d; ++q) {
            double avg = 0.0;
            for (int j = 0; j < r; ++j) avg += p[j] * phi[(long)j * d + q];
            xi[q] = gx[q] - phi[(long)k * d + q] + avg;
        }
        for (long q = 0; q < d; ++q) v[q] = x[q] - tau * xi[q];
        orc_prox(n, reg_kind, tau, lam, tv_w, tv_eps, tv_inner, v, x, tvd, xn);
        for (long e = 0; e < m; ++e) {
            const double zeta = dd[e] + psibar[e];
            y[e] = (y[e] + sigma * zeta - sigma * bdata[e]) / (1.0 + sigma);
            psibar[e] += p[k] * dd[e];
        }
        memcpy(zsnap + (long)k * d, x, sizeof(double) * d);
        memcpy(x, xn, sizeof(double) * d);
        memcpy(phi + (long)k * d, gx, sizeof(double) * d);
        if (draws_out) draws_out[it] = k;
        if (epochs) {
            if (k == 0 && mode == ORC_MODE_UNBIASED) *epochs += unbiased_full;
            else *epochs += ldexp(1.0, -log2f[k]);
        }
    }
    free(gx);
    free(dd);
    free(diff);
    free(xi);
    free(xn);
    free(v);
    free(idx);
    return 0;
}

/* Alg. 1 with independent primal and dual sketch draws (the first item of
 * the paper's outlook, Sec. 6): the primal index i_k comes from stream
 * `stream`, the dual index j_k from stream `dual_stream` (same seed and p).
 * The dual step refreshes psi_{j_k} from K_{j_k} x^k, the primal step
 * phi_{i_k} from K_{i_k}^T y^k; both from the old iterates, old-table
 * averages.  An iteration costs half of each side's level cost:
 * epochs += (c(i_k) + c(j_k)) / 2, so equal streams reproduce orc_imask_run.
 * draws_out gets i_k, dual_draws_out j_k (either may be NULL). */
int orc_imask_indep_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                        int r, const int* log2f, const double* p, int mode,
                        int reg_kind, double lam, double tv_w, double tv_eps, int tv_inner,
                        double sigma, uint64_t seed, uint32_t stream, uint32_t dual_stream, uint64_t k0,
                        const double* bdata, int n_iter,
                        double* x, double* y, double* phi, double* psi, double* tvd,
                        int32_t* draws_out, int32_t* dual_draws_out, double* epochs)
{
    if (r < 1 || r > ORC_MAX_LEVELS || log2f[0] != 0) return -1;
    const long d = (long)n * n, m = (long)na * nd;
    const double tau = sigma / lam;
    double* gx = (double*)malloc(sizeof(double) * d);
    double* gy = (double*)malloc(sizeof(double) * m);
    double* xn = (double*)malloc(sizeof(double) * d);
    double* v = (double*)malloc(sizeof(double) * d);
    int32_t* ip = (int32_t*)malloc(sizeof(int32_t) * (n_iter > 0 ? n_iter : 1));
    int32_t* jd = (int32_t*)malloc(sizeof(int32_t) * (n_iter > 0 ? n_iter : 1));
    orc_draws(seed, stream, k0, n_iter, r, p, ip);
    orc_draws(seed, dual_stream, k0, n_iter, r, p, jd);
    double cost[ORC_MAX_LEVELS];
    for (int k = 0; k < r; ++k) cost[k] = ldexp(1.0, -log2f[k]);
    if (mode == ORC_MODE_UNBIASED)
        for (int k = 1; k < r; ++k) cost[0] += ldexp(1.0, -log2f[k]);
    for (int it = 0; it < n_iter; ++it) {
        const int i = ip[it], j = jd[it];
        orc_sketch_adj(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, i, y, gx);
        orc_sketch_fwd(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, j, x, gy);
        for (long q = 0; q < d; ++q) {
            double avg = 0.0;
            for (int c = 0; c < r; ++c) avg += p[c] * phi[(long)c * d + q];
            v[q] = x[q] - tau * (gx[q] - phi[(long)i * d + q] + avg);
        }
        orc_prox(n, reg_kind, tau, lam, tv_w, tv_eps, tv_inner, v, x, tvd, xn);
        for (long e = 0; e < m; ++e) {
            double avg = 0.0;
            for (int c = 0; c < r; ++c) avg += p[c] * psi[(long)c * m + e];
            const double zeta = gy[e] - psi[(long)j * m + e] + avg;
            y[e] = (y[e] + sigma * zeta - sigma * bdata[e]) / (1.0 + sigma);
        }
        memcpy(x, xn, sizeof(double) * d);
        memcpy(phi + (long)i * d, gx, sizeof(double) * d);
        memcpy(psi + (long)j * m, gy, sizeof(double) * m);
        if (draws_out) draws_out[it] = i;
        if (dual_draws_out) dual_draws_out[it] = j;
        if (epochs) *epochs += 0.5 * (cost[i] + cost[j]);
    }
    free(gx);
    free(gy);
    free(xn);
    free(v);
    free(ip);
    free(jd);
    return 0;
}


/* ------------------------------------------------------ measurement blocks */

/* Image sketches combined with measurement sub-selection (the paper's
 * outlook, Sec. 6), read as Alg. 1 over the product family
 *   K_{ij} = S E_j K_i,   i ~ p,  j uniform over S blocks (q_j = 1/S),
 * with E_j keeping the rows of angle block j = [floor(j na/S),
 * floor((j+1) na/S)) and zeroing the others, so sum_ij p_i q_j K_ij =
 * sum_i p_i K_i.  Block j of draw k comes from the low word of the same
 * SplitMix64 output whose high word picks i: j = (lo32 * S) >> 32.
 * Tables: phi_{ij} = K_ij^T y (one full image per pair, index i S + j);
 * psi_i holds K_ij x on the rows of every block j (one m-table per i).
 * The dual estimate is dense: zeta = E_j (K_ij x - psi_i) + sum_i' p_i'/S
 * psi_i' on every row; only block j's rows of psi_i are refreshed.
 * A step costs c(i) (a1 - a0) / na epochs.  S = 1 is Alg. 1. */
void orc_block_rows(int na, int S, int j, int* a0, int* a1)
{
    *a0 = (int)(((long)j * na) / S);
    *a1 = (int)(((long)(j + 1) * na) / S);
}

void orc_block_draws(uint64_t seed, uint32_t stream, uint64_t k0, int count, int S, int32_t* out)
{
    const uint64_t ss = orc_splitmix64(seed, stream);
    for (int q = 0; q < count; ++q) {
        const uint64_t lo = orc_splitmix64(ss, k0 + (uint64_t)q) & 0xffffffffULL;
        out[q] = (int32_t)((lo * (uint64_t)S) >> 32);
    }
}

int orc_imask_blocks_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                         int r, const int* log2f, const double* p, int mode, int S,
                         int reg_kind, double lam, double tv_w, double tv_eps, int tv_inner,
                         double sigma, uint64_t seed, uint32_t stream, uint64_t k0,
                         const double* bdata, int n_iter,
                         double* x, double* y, double* phi, double* psi, double* tvd,
                         int32_t* draws_out, int32_t* blocks_out, double* epochs)
{
    if (r < 1 || r > ORC_MAX_LEVELS || log2f[0] != 0 || S < 1 || S > na) return -1;
    const long d = (long)n * n, m = (long)na * nd;
    const double tau = sigma / lam;
    double* gx = (double*)malloc(sizeof(double) * d);
    double* gy = (double*)malloc(sizeof(double) * m);
    double* yj = (double*)malloc(sizeof(double) * m);
    double* xi = (double*)malloc(sizeof(double) * d);
    double* zeta = (double*)malloc(sizeof(double) * m);
    double* xn = (double*)malloc(sizeof(double) * d);
    double* v = (double*)malloc(sizeof(double) * d);
    const int cnt = n_iter > 0 ? n_iter : 1;
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * cnt);
    int32_t* jdx = (int32_t*)malloc(sizeof(int32_t) * cnt);
    orc_draws(seed, stream, k0, n_iter, r, p, idx);
    orc_block_draws(seed, stream, k0, n_iter, S, jdx);
    double unbiased_full = 1.0;
    for (int k = 1; k < r; ++k) unbiased_full += ldexp(1.0, -log2f[k]);
    for (int it = 0; it < n_iter; ++it) {
        const int k = idx[it], j = jdx[it];
        int a0, a1;
        orc_block_rows(na, S, j, &a0, &a1);
        const long e0 = (long)a0 * nd, e1 = (long)a1 * nd;
        /* K_kj^T y = S K_k^T E_j y and K_kj x = S E_j K_k x, old iterates */
        for (long e = 0; e < m; ++e) yj[e] = (e >= e0 && e < e1) ? y[e] : 0.0;
        orc_sketch_adj(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, yj, gx);
        for (long q = 0; q < d; ++q) gx[q] *= S;
        orc_sketch_fwd(n, na, nd, ds, s0, E, ang, D, Dd, r, log2f, p, mode, k, x, gy);
        for (long e = 0; e < m; ++e) gy[e] = (e >= e0 && e < e1) ? S * gy[e] : 0.0;
        /* SAGA estimates with the old tables */
        for (long q = 0; q < d; ++q) {
            double avg = 0.0;
            for (int c = 0; c < r; ++c)
                for (int b = 0; b < S; ++b) avg += p[c] / S * phi[((long)c * S + b) * d + q];
            xi[q] = gx[q] - phi[((long)k * S + j) * d + q] + avg;
        }
        for (long e = 0; e < m; ++e) {
            double avg = 0.0;
            for (int c = 0; c < r; ++c) avg += p[c] / S * psi[(long)c * m + e];
            zeta[e] = (e >= e0 && e < e1) ? gy[e] - psi[(long)k * m + e] + avg : avg;
        }
        for (long q = 0; q < d; ++q) v[q] = x[q] - tau * xi[q];
        orc_prox(n, reg_kind, tau, lam, tv_w, tv_eps, tv_inner, v, x, tvd, xn);
        for (long e = 0; e < m; ++e) y[e] = (y[e] + sigma * zeta[e] - sigma * bdata[e]) / (1.0 + sigma);
        memcpy(x, xn, sizeof(double) * d);
        memcpy(phi + ((long)k * S + j) * d, gx, sizeof(double) * d);
        memcpy(psi + (long)k * m + e0, gy + e0, sizeof(double) * (e1 - e0));
        if (draws_out) draws_out[it] = k;
        if (blocks_out) blocks_out[it] = j;
        if (epochs) {
            const double c = (k == 0 && mode == ORC_MODE_UNBIASED) ? unbiased_full : ldexp(1.0, -log2f[k]);
            *epochs += c * (double)(a1 - a0) / na;
        }
    }
    free(gx);
    free(gy);
    free(yj);
    free(xi);
    free(zeta);
    free(xn);
    free(v);
    free(idx);
    free(jdx);
    return 0;
}
