/* Drives every entry point of the FP64 oracle (oracle/imask_oracle.c) on
 * small seeded inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitize_cpu.py).  It also checks
 * the adjoint identity <A z, y> = <z, A^T y> of the projector pair and of
 * the sketches, so a run that only "does not crash" still computes.  Exit
 * status 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_project(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd, int lvl,
                 const double* z, double* sino);
void orc_backproject(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                     int lvl, const double* sino, double* z);
long long orc_count_samples(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D,
                            double Dd, int lvl);
void orc_restrict(int n, int lvl, const double* x, double* z);
void orc_prolong(int n, int lvl, const double* z, double* x);
void orc_compensate(int n, int r, const int* log2f, const double* p, const double* x, double* out);
void orc_sketch_fwd(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                    int r, const int* log2f, const double* p, int mode, int k, const double* x, double* g);
void orc_sketch_adj(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                    int r, const int* log2f, const double* p, int mode, int k, const double* y, double* g);
void orc_draws(uint64_t seed, uint32_t stream, uint64_t k0, int count, int r, const double* p, int32_t* out);
void orc_block_draws(uint64_t seed, uint32_t stream, uint64_t k0, int count, int S, int32_t* out);
double orc_tv_value(int n, const double* u, double eps);
void orc_tv_gradient(int n, const double* u, double eps, double* out);
void orc_tv_prox(int n, const double* v, const double* u0, double tau, double lam, double w, double eps, int J,
                 double* out);
void orc_tv_fgp(int n, const double* b, double gamma, int J, double* p1, double* p2, double* u);
int orc_imask_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd, int r,
                  const int* log2f, const double* p, int mode, int reg_kind, double lam, double tv_w, double tv_eps,
                  int tv_inner, double sigma, uint64_t seed, uint32_t stream, uint64_t k0, const double* bdata,
                  int n_iter, double* x, double* y, double* phi, double* psi, double* tvd, int32_t* draws_out,
                  double* epochs);
int orc_imask_seq_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                      int r, const int* log2f, const double* p, int mode, int reg_kind, double lam, double tv_w,
                      double tv_eps, int tv_inner, double sigma, double theta, uint64_t seed, uint32_t stream,
                      uint64_t k0, const double* bdata, int n_iter, double* x, double* xbar, double* y, double* phi,
                      double* psi, double* tvd, int32_t* draws_out, double* epochs);
int orc_imask_compact_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D,
                          double Dd, int r, const int* log2f, const double* p, int mode, int reg_kind, double lam,
                          double tv_w, double tv_eps, int tv_inner, double sigma, uint64_t seed, uint32_t stream,
                          uint64_t k0, const double* bdata, int n_iter, double* x, double* y, double* phi,
                          double* zsnap, double* psibar, double* tvd, int32_t* draws_out, double* epochs);
int orc_imask_indep_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D, double Dd,
                        int r, const int* log2f, const double* p, int mode, int reg_kind, double lam, double tv_w,
                        double tv_eps, int tv_inner, double sigma, uint64_t seed, uint32_t stream,
                        uint32_t dual_stream, uint64_t k0, const double* bdata, int n_iter, double* x, double* y,
                        double* phi, double* psi, double* tvd, int32_t* draws_out, int32_t* dual_draws_out,
                        double* epochs);
int orc_imask_blocks_run(int n, int na, int nd, double ds, double s0, double E, const double* ang, double D,
                         double Dd, int r, const int* log2f, const double* p, int mode, int S, int reg_kind,
                         double lam, double tv_w, double tv_eps, int tv_inner, double sigma, uint64_t seed,
                         uint32_t stream, uint64_t k0, const double* bdata, int n_iter, double* x, double* y,
                         double* phi, double* psi, double* tvd, int32_t* draws_out, int32_t* blocks_out,
                         double* epochs);

static uint64_t rng = 0x9E3779B97F4A7C15ULL;
static double urand(void)  /* xorshift64*, in [-1, 1) */
{
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return (double)((rng * 2685821657736338717ULL) >> 11) / 4503599627370496.0 - 1.0;
}
static double* vec(long n)
{
    double* v = (double*)malloc(sizeof(double) * (size_t)n);
    for (long q = 0; q < n; ++q) v[q] = urand();
    return v;
}
static double dot(const double* a, const double* b, long n)
{
    double s = 0.0;
    for (long q = 0; q < n; ++q) s += a[q] * b[q];
    return s;
}
static int fails = 0;
static void check_adjoint(const char* what, double lhs, double rhs)
{
    const double err = fabs(lhs - rhs) / (fabs(lhs) + fabs(rhs) + 1e-300);
    if (err > 1e-12) {
        printf("%s: adjoint mismatch %.3e\n", what, err);
        ++fails;
    }
}

int main(void)
{
    /* parallel beam (default angles and a listed set) and a fan beam */
    const int n = 16, na = 12, nd = 26;
    const double E = 1.0, ds = 2.0 * E / n, s0 = 0.05;
    double ang[12];
    for (int a = 0; a < na; ++a) ang[a] = 0.37 * a - 1.1;
    struct {
        const double* ang;
        double D, Dd;
    } geo[3] = {{NULL, 0.0, 0.0}, {ang, 0.0, 0.0}, {NULL, 4.0, 2.0}};
    const long d = (long)n * n, m = (long)na * nd;
    for (int gi = 0; gi < 3; ++gi) {
        for (int lvl = 0; lvl <= 3; ++lvl) {
            const long dl = (long)(n >> lvl) * (n >> lvl);
            double *z = vec(dl), *y = vec(m), *Az = calloc(m, sizeof(double)), *Aty = calloc(dl, sizeof(double));
            orc_project(n, na, nd, ds, s0, E, geo[gi].ang, geo[gi].D, geo[gi].Dd, lvl, z, Az);
            orc_backproject(n, na, nd, ds, s0, E, geo[gi].ang, geo[gi].D, geo[gi].Dd, lvl, y, Aty);
            check_adjoint("projector", dot(Az, y, m), dot(z, Aty, dl));
            if (orc_count_samples(n, na, nd, ds, s0, E, geo[gi].ang, geo[gi].D, geo[gi].Dd, lvl) <= 0) ++fails;
            free(z), free(y), free(Az), free(Aty);
        }
    }
    /* resampling, compensation, sketches in both modes */
    const int r = 3, log2f[3] = {0, 1, 2};
    const double p[3] = {0.5, 0.3, 0.2};
    {
        double *x = vec(d), *z = calloc(d, sizeof(double)), *x2 = calloc(d, sizeof(double));
        orc_restrict(n, 2, x, z);
        orc_prolong(n, 2, z, x2);
        orc_compensate(n, r, log2f, p, x, x2);
        for (int mode = 0; mode < 2; ++mode)
            for (int k = 0; k < r; ++k) {
                double *xs = vec(d), *y = vec(m), *g = calloc(m, sizeof(double)), *h = calloc(d, sizeof(double));
                orc_sketch_fwd(n, na, nd, ds, s0, E, NULL, 0.0, 0.0, r, log2f, p, mode, k, xs, g);
                orc_sketch_adj(n, na, nd, ds, s0, E, NULL, 0.0, 0.0, r, log2f, p, mode, k, y, h);
                check_adjoint("sketch", dot(g, y, m), dot(xs, h, d));
                free(xs), free(y), free(g), free(h);
            }
        free(x), free(z), free(x2);
    }
    /* draws, TV pieces */
    {
        int32_t dr[64], bl[64];
        orc_draws(42, 7, 100, 64, r, p, dr);
        orc_block_draws(42, 7, 100, 64, 4, bl);
        for (int q = 0; q < 64; ++q)
            if (dr[q] < 0 || dr[q] >= r || bl[q] < 0 || bl[q] >= 4) ++fails;
        double *u = vec(d), *v = vec(d), *g = calloc(d, sizeof(double)), *o = calloc(d, sizeof(double));
        double *p1 = calloc(d, sizeof(double)), *p2 = calloc(d, sizeof(double));
        if (!(orc_tv_value(n, u, 1e-2) >= 0.0)) ++fails;
        orc_tv_gradient(n, u, 1e-2, g);
        orc_tv_prox(n, v, u, 0.1, 0.5, 0.2, 1e-2, 5, o);
        orc_tv_fgp(n, v, 0.1, 5, p1, p2, o);
        free(u), free(v), free(g), free(o), free(p1), free(p2);
    }
    /* a few iterations of every solver variant, every prior */
    double* b = vec(m);
    for (int reg = 0; reg < 3; ++reg)
        for (int mode = 0; mode < 2; ++mode) {
            double *x = calloc(d, sizeof(double)), *xb = calloc(d, sizeof(double)), *y = calloc(m, sizeof(double));
            double *phi = calloc(r * d, sizeof(double)), *psi = calloc(r * m, sizeof(double));
            double *tvd = calloc(2 * d, sizeof(double)), *zs = calloc(r * d, sizeof(double));
            double* pb = calloc(m, sizeof(double));
            double *phiB = calloc(4 * r * d, sizeof(double)), *psiB = calloc(r * m, sizeof(double));
            int32_t dr[8], dd[8], bl[8];
            double ep = 0.0;
            fails += orc_imask_run(n, na, nd, ds, s0, E, NULL, 0.0, 0.0, r, log2f, p, mode, reg, 0.5, 0.05, 1e-2, 4,
                                   1e-2, 42, 3, 0, b, 6, x, y, phi, psi, tvd, dr, &ep) != 0;
            fails += orc_imask_seq_run(n, na, nd, ds, s0, E, NULL, 0.0, 0.0, r, log2f, p, mode, reg, 0.5, 0.05, 1e-2,
                                       4, 1e-2, 1.0, 42, 3, 0, b, 6, x, xb, y, phi, psi, tvd, dr, &ep) != 0;
            fails += orc_imask_compact_run(n, na, nd, ds, s0, E, NULL, 0.0, 0.0, r, log2f, p, mode, reg, 0.5, 0.05,
                                           1e-2, 4, 1e-2, 42, 3, 0, b, 6, x, y, phi, zs, pb, tvd, dr, &ep) != 0;
            fails += orc_imask_indep_run(n, na, nd, ds, s0, E, NULL, 4.0, 2.0, r, log2f, p, mode, reg, 0.5, 0.05,
                                         1e-2, 4, 1e-2, 42, 3, 5, 0, b, 6, x, y, phi, psi, tvd, dr, dd, &ep) != 0;
            fails += orc_imask_blocks_run(n, na, nd, ds, s0, E, NULL, 0.0, 0.0, r, log2f, p, mode, 4, reg, 0.5, 0.05,
                                          1e-2, 4, 1e-2, 42, 3, 0, b, 6, x, y, phiB, psiB, tvd, dr, bl, &ep) != 0;
            for (long q = 0; q < d; ++q)
                if (!isfinite(x[q])) {
                    ++fails;
                    break;
                }
            free(x), free(xb), free(y), free(phi), free(psi), free(tvd), free(zs), free(pb), free(phiB), free(psiB);
        }
    free(b);
    printf(fails ? "FAILED %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
