// api.hip - the C ABI of libimask (include/imask.h): argument validation,
// workspace layout, the host-side sketch draw and the per-step launch
// sequence of Alg. 1.  All device work goes to the caller's stream; no call
// allocates, frees or synchronises.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "imask.h"
#include "internal.h"

namespace imk {

static size_t align64(size_t f) { return (f + 63) & ~(size_t)63; }

static int level_limit(int n)
{
    int l = 0;
    while (l < IMASK_MAX_LOG2F && (n % (2 << l)) == 0 && (n >> (l + 1)) >= 2) ++l;
    return l;
}

Layout make_layout(const imask_geometry& g)
{
    Layout L;
    L.n = g.n;
    L.na = g.n_angles;
    L.nd = g.n_det;
    L.lmax = level_limit(g.n);
    size_t off = 0;
    L.consts = off;
    off = align64(off + (size_t)(L.lmax + 1) * g.n_angles * kConstStride);
    for (int l = 0; l <= L.lmax; ++l) {
        const size_t pad = (size_t)side(g.n, l) * pstride(g.n, l);
        L.zp[l] = off;
        off = align64(off + pad);
        L.zpT[l] = off;
        off = align64(off + pad);
        L.craw[l] = off;
        off = align64(off + (size_t)side(g.n, l) * side(g.n, l));
    }
    L.vbuf = off;
    off = align64(off + (size_t)g.n * g.n);
    L.part = off;
    off = align64(off + (size_t)16 * g.n * g.n);
    L.ptmp = off;
    off = align64(off + (size_t)g.n * g.n);
    const size_t m = (size_t)g.n_angles * g.n_det;
    for (int l = 0; l <= L.lmax; ++l) {
        fwd_bands(side(g.n, l), &L.fbands[l], &L.frows[l]);
        L.fpart[l] = off;
        off = align64(off + (size_t)L.fbands[l] * m);
    }
    L.total = off;
    return L;
}

// ---- validation ----

static bool geometry_ok(const imask_geometry* g)
{
    if (!g) return false;
    if (g->n < 4 || g->n > 16384 || (g->n % 4) != 0) return false;
    if (g->n > 16 && (g->n % 16) != 0) return false;
    if (g->n_angles < 1 || g->n_det < 1 || g->n_angles > 65536 || g->n_det > 8192) return false;
    if (!std::isfinite(g->det_spacing) || !std::isfinite(g->det_offset)) return false;
    return true;
}

static bool levels_ok(const imask_levels* lv, int lmax)
{
    if (!lv || lv->r < 1 || lv->r > IMASK_MAX_LEVELS) return false;
    if (lv->log2f[0] != 0) return false;
    double sum = 0.0;
    for (int k = 0; k < lv->r; ++k) {
        if (k > 0 && lv->log2f[k] <= lv->log2f[k - 1]) return false;
        if (lv->log2f[k] > lmax) return false;
        if (!(lv->p[k] > 0.0) || !std::isfinite(lv->p[k])) return false;
        sum += lv->p[k];
    }
    if (std::fabs(sum - 1.0) > 1e-9) return false;
    return lv->full_mode == IMASK_FULL_PAPER || lv->full_mode == IMASK_FULL_UNBIASED;
}

static bool reg_ok(const imask_reg* r)
{
    if (!r || !(r->lambda > 0.0) || !std::isfinite(r->lambda)) return false;
    if (r->kind == IMASK_REG_TIKHONOV) return true;
    if (r->kind != IMASK_REG_SMOOTH_TV) return false;
    return r->tv_weight >= 0.0 && std::isfinite(r->tv_weight) && r->tv_eps > 0.0 && std::isfinite(r->tv_eps) &&
           r->tv_inner >= 1 && r->tv_inner <= IMASK_MAX_TV_INNER;
}

static bool state_ok(const imask_state* s)
{
    return s && s->x[0] && s->x[1] && s->y[0] && s->y[1] && s->phi && s->psi && s->work &&
           (s->cur == 0 || s->cur == 1) && s->x[0] != s->x[1] && s->y[0] != s->y[1];
}

// ---- sketch draw: SplitMix64 (Steele, Lea & Flood 2014), counter form ----

static inline uint64_t mix_at(uint64_t state0, uint64_t k)
{
    uint64_t z = state0 + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static void draw_thresholds(const imask_levels& lv, uint64_t* thr)
{
    double cum = 0.0;
    for (int j = 0; j < lv.r; ++j) {
        cum += lv.p[j];
        double t = std::floor(4294967296.0 * cum);
        if (t > 4294967296.0) t = 4294967296.0;
        thr[j] = (uint64_t)t;
    }
    thr[lv.r - 1] = 4294967296ULL;
}

static int draw_one(const imask_params& prm, const uint64_t* thr, uint64_t k)
{
    const uint64_t stream_state = mix_at(prm.seed, prm.stream_id);
    const uint64_t u = mix_at(stream_state, k) >> 32;
    int j = 0;
    while (u >= thr[j]) ++j;
    return j;
}

static double sketch_cost(const imask_levels& lv, int k)
{
    if (k == 0 && lv.full_mode == IMASK_FULL_UNBIASED) {
        double c = 1.0;
        for (int j = 1; j < lv.r; ++j) c += std::ldexp(1.0, -lv.log2f[j]);
        return c;
    }
    return std::ldexp(1.0, -lv.log2f[k]);
}

// ---- launch building blocks ----

#define IMK_TRY(expr)                                 \
    do {                                              \
        if ((expr) != hipSuccess) return IMASK_EHIP;  \
    } while (0)

// Restricted / compensated copies of x for the forward of sketch k, and the
// projector terms that combine them into K_k x.
static void forward_plan(const Layout& L, const imask_levels& lv, int k, const float* x, float* W,
                         PrepArgs& pa, FwdArgs& fa)
{
    const int lmax_set = lv.log2f[lv.r - 1];
    pa = PrepArgs{};
    pa.x = x;
    pa.n = L.n;
    pa.T = tile_side(L.n, lmax_set);
    fa.nterms = 0;
    if (k > 0) {
        const int l = lv.log2f[k];
        pa.out[0] = PrepOut{W + L.zp[l], W + L.zpT[l], l, PREP_MEAN, 1};
        pa.nout = 1;
        pa.pyr_levels = l;
        fa.term[0] = FwdTerm{W + L.zp[l], W + L.zpT[l], l, 1.0f, W + L.fpart[l], L.fbands[l], L.frows[l]};
        fa.nterms = 1;
    } else if (lv.r == 1 || lv.full_mode == IMASK_FULL_PAPER) {
        pa.out[0] = PrepOut{W + L.zp[0], W + L.zpT[0], 0, lv.r > 1 ? PREP_COMP : PREP_MEAN, 1};
        pa.nout = 1;
        pa.pyr_levels = lv.r > 1 ? lmax_set : 0;
        pa.ncomp = lv.r - 1;
        for (int j = 1; j < lv.r; ++j) {
            pa.comp_lvl[j - 1] = lv.log2f[j];
            pa.comp_p[j - 1] = (float)lv.p[j];
        }
        pa.inv_p0 = (float)(1.0 / lv.p[0]);
        fa.term[0] = FwdTerm{W + L.zp[0], W + L.zpT[0], 0, 1.0f, W + L.fpart[0], L.fbands[0], L.frows[0]};
        fa.nterms = 1;
    } else {
        pa.nout = lv.r;
        pa.pyr_levels = lmax_set;
        for (int j = 0; j < lv.r; ++j) {
            const int l = lv.log2f[j];
            pa.out[j] = PrepOut{W + L.zp[l], W + L.zpT[l], l, PREP_MEAN, 1};
            const float coef = (float)(j == 0 ? 1.0 / lv.p[0] : -lv.p[j] / lv.p[0]);
            fa.term[j] = FwdTerm{W + L.zp[l], W + L.zpT[l], l, coef, W + L.fpart[l], L.fbands[l], L.frows[l]};
        }
        fa.nterms = lv.r;
    }
}

static void fwd_common(const Layout& L, const float* W, FwdArgs& fa)
{
    fa.consts = (const RayConst*)(W + L.consts);
    fa.n = L.n;
    fa.na = L.na;
    fa.nd = L.nd;
}

static int backproject_raw(const Layout& L, const float* W, int lvl, const float* y, float* out, float coef,
                           int accumulate, int prolong, hipStream_t s)
{
    BpArgs ba{};
    ba.consts = (const RayConst*)(W + L.consts);
    ba.n = L.n;
    ba.na = L.na;
    ba.nd = L.nd;
    ba.lvl = lvl;
    ba.y = y;
    ba.out = out;
    ba.coef = coef;
    ba.accumulate = accumulate;
    ba.prolong = prolong;
    ba.part = const_cast<float*>(W) + L.part;
    ba.tmp = const_cast<float*>(W) + L.ptmp;
    IMK_TRY(launch_bp(ba, s));
    return IMASK_OK;
}

static void phi_offsets(const imask_geometry& g, const imask_levels& lv, long long* off)
{
    long long o = 0;
    for (int k = 0; k < lv.r; ++k) {
        off[k] = o;
        const long long nl = g.n >> lv.log2f[k];
        o += nl * nl;
    }
}

static int one_step(const imask_geometry& g, const Layout& L, const imask_levels& lv, const imask_reg& reg,
                    const imask_params& prm, const float* bdat, imask_state& st, hipStream_t s)
{
    uint64_t thr[IMASK_MAX_LEVELS];
    draw_thresholds(lv, thr);
    const int k = draw_one(prm, thr, st.k);
    float* W = (float*)st.work;
    const int cur = st.cur, nxt = 1 - cur;
    const int lmax_set = lv.log2f[lv.r - 1];

    // a2-a4: restriction, forward projection, dual SAGA step and psi refresh
    PrepArgs pa;
    FwdArgs fa{};
    forward_plan(L, lv, k, st.x[cur], W, pa, fa);
    fwd_common(L, W, fa);
    fa.mode = FWD_DUAL;
    fa.y_old = st.y[cur];
    fa.y_new = st.y[nxt];
    fa.bdat = bdat;
    fa.psi = st.psi;
    fa.r = lv.r;
    fa.kidx = k;
    for (int j = 0; j < lv.r; ++j) fa.p[j] = (float)lv.p[j];
    fa.sigma = (float)prm.sigma;
    fa.inv1ps = (float)(1.0 / (1.0 + prm.sigma));
    IMK_TRY(launch_prep(pa, s));
    IMK_TRY(launch_fwd(fa, s));

    // a5: raw backprojections R_l^T y^k needed by sketch k
    if (k > 0) {
        const int l = lv.log2f[k];
        if (int rc = backproject_raw(L, W, l, st.y[cur], W + L.craw[l], 1.0f, 0, 0, s)) return rc;
    } else {
        if (int rc = backproject_raw(L, W, 0, st.y[cur], W + L.craw[0], 1.0f, 0, 0, s)) return rc;
        if (lv.full_mode == IMASK_FULL_UNBIASED)
            for (int j = 1; j < lv.r; ++j) {
                const int l = lv.log2f[j];
                if (int rc = backproject_raw(L, W, l, st.y[cur], W + L.craw[l], 1.0f, 0, 0, s)) return rc;
            }
    }

    // a6-a7: prolongation / compensation, primal SAGA step, phi refresh
    const double tau = prm.sigma / reg.lambda;
    const bool tv = reg.kind == IMASK_REG_SMOOTH_TV;
    PrimalArgs pr{};
    pr.n = g.n;
    pr.T = tile_side(g.n, lmax_set);
    pr.pyr_levels = lmax_set;
    pr.r = lv.r;
    pr.kidx = k;
    pr.full_mode = lv.full_mode;
    for (int j = 0; j < lv.r; ++j) {
        pr.lvl[j] = lv.log2f[j];
        pr.p[j] = (float)lv.p[j];
        pr.craw[j] = W + L.craw[lv.log2f[j]];
    }
    pr.phi = st.phi;
    phi_offsets(g, lv, pr.phi_off);
    pr.x_old = st.x[cur];
    pr.x_out = tv ? W + L.vbuf : st.x[nxt];
    pr.tau = (float)tau;
    pr.prox_scale = tv ? 1.0f : (float)(1.0 / (1.0 + tau * reg.lambda));
    IMK_TRY(launch_primal(pr, s));

    // a8: smoothed-TV prox by FISTA, warm-started at x^k
    if (tv) {
        TvArgs ta{};
        ta.n = g.n;
        ta.J = reg.tv_inner;
        ta.v = W + L.vbuf;
        ta.u0 = st.x[cur];
        ta.out = st.x[nxt];
        ta.tau_w = (float)(tau * reg.tv_weight);
        ta.tau_lam = (float)(tau * reg.lambda);
        ta.eps = (float)reg.tv_eps;
        ta.invL = (float)(1.0 / (1.0 + tau * reg.lambda + 8.0 * tau * reg.tv_weight / reg.tv_eps));
        double t = 1.0;
        for (int it = 0; it < reg.tv_inner; ++it) {
            const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
            ta.beta[it] = (float)((t - 1.0) / tn);
            t = tn;
        }
        IMK_TRY(launch_tv(ta, s));
    }

    st.cur = nxt;
    st.k += 1;
    st.epochs += sketch_cost(lv, k);
    return IMASK_OK;
}

}  // namespace imk

using namespace imk;

extern "C" {

size_t imask_workspace_bytes(const imask_geometry* g)
{
    if (!geometry_ok(g)) return 0;
    return make_layout(*g).total * sizeof(float);
}

size_t imask_phi_floats(const imask_geometry* g, const imask_levels* lv)
{
    if (!geometry_ok(g) || !levels_ok(lv, level_limit(g->n))) return 0;
    size_t t = 0;
    for (int k = 0; k < lv->r; ++k) {
        const size_t nl = (size_t)(g->n >> lv->log2f[k]);
        t += nl * nl;
    }
    return t;
}

int imask_prepare(const imask_geometry* g, void* work, size_t work_bytes, void* stream)
{
    if (!geometry_ok(g) || !work) return IMASK_EINVAL;
    const Layout L = make_layout(*g);
    if (work_bytes < L.total * sizeof(float)) return IMASK_ESIZE;
    hipStream_t s = (hipStream_t)stream;
    IMK_TRY(launch_fill((float*)work, L.total, 0.0f, s));
    IMK_TRY(launch_consts(*g, L, (float*)work, s));
    return IMASK_OK;
}

int imask_project(const imask_geometry* g, int32_t log2f, const void* work, const float* x_full, float* sino,
                  void* stream)
{
    if (!geometry_ok(g) || !work || !x_full || !sino) return IMASK_EINVAL;
    const Layout L = make_layout(*g);
    if (log2f < 0 || log2f > L.lmax) return IMASK_EINVAL;
    float* W = (float*)work;
    hipStream_t s = (hipStream_t)stream;
    PrepArgs pa{};
    pa.x = x_full;
    pa.n = g->n;
    pa.T = tile_side(g->n, log2f);
    pa.pyr_levels = log2f;
    pa.nout = 1;
    pa.out[0] = PrepOut{W + L.zp[log2f], W + L.zpT[log2f], log2f, PREP_MEAN, 1};
    FwdArgs fa{};
    fwd_common(L, W, fa);
    fa.nterms = 1;
    fa.term[0] = FwdTerm{W + L.zp[log2f], W + L.zpT[log2f], log2f, 1.0f, W + L.fpart[log2f], L.fbands[log2f],
                         L.frows[log2f]};
    fa.mode = FWD_STORE;
    fa.out = sino;
    IMK_TRY(launch_prep(pa, s));
    IMK_TRY(launch_fwd(fa, s));
    return IMASK_OK;
}

int imask_backproject(const imask_geometry* g, int32_t log2f, const void* work, const float* sino, float* x_full,
                      void* stream)
{
    if (!geometry_ok(g) || !work || !sino || !x_full) return IMASK_EINVAL;
    const Layout L = make_layout(*g);
    if (log2f < 0 || log2f > L.lmax) return IMASK_EINVAL;
    return backproject_raw(L, (const float*)work, log2f, sino, x_full, 1.0f / (float)(1 << (2 * log2f)), 0, 1,
                           (hipStream_t)stream);
}

int imask_resample(int32_t n, int32_t log2f, int32_t mode, const imask_levels* lv, const float* in, float* out,
                   void* stream)
{
    imask_geometry g{n, 1, 1, 0.0, 0.0};
    if (!geometry_ok(&g) || !in || !out || in == out) return IMASK_EINVAL;
    const int lmax = level_limit(n);
    if (log2f < 0 || log2f > lmax) return IMASK_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    switch (mode) {
    case IMASK_RESTRICT: {
        PrepArgs pa{};
        pa.x = in;
        pa.n = n;
        pa.T = tile_side(n, log2f);
        pa.pyr_levels = log2f;
        pa.nout = 1;
        pa.out[0] = PrepOut{out, nullptr, log2f, PREP_MEAN, 0};
        IMK_TRY(launch_prep(pa, s));
        return IMASK_OK;
    }
    case IMASK_PROLONG:
        IMK_TRY(launch_prolong(in, out, n, log2f, 1.0f, s));
        return IMASK_OK;
    case IMASK_RESTRICT_ADJ:
        IMK_TRY(launch_prolong(in, out, n, log2f, 1.0f / (float)(1 << (2 * log2f)), s));
        return IMASK_OK;
    case IMASK_PROJECT:
        IMK_TRY(launch_project_block(in, out, n, log2f, s));
        return IMASK_OK;
    case IMASK_COMPENSATE: {
        if (!levels_ok(lv, lmax)) return IMASK_EINVAL;
        PrepArgs pa{};
        pa.x = in;
        pa.n = n;
        pa.T = tile_side(n, lv->log2f[lv->r - 1]);
        pa.pyr_levels = lv->log2f[lv->r - 1];
        pa.nout = 1;
        pa.out[0] = PrepOut{out, nullptr, 0, lv->r > 1 ? PREP_COMP : PREP_MEAN, 0};
        pa.ncomp = lv->r - 1;
        for (int j = 1; j < lv->r; ++j) {
            pa.comp_lvl[j - 1] = lv->log2f[j];
            pa.comp_p[j - 1] = (float)lv->p[j];
        }
        pa.inv_p0 = (float)(1.0 / lv->p[0]);
        IMK_TRY(launch_prep(pa, s));
        return IMASK_OK;
    }
    default:
        return IMASK_EINVAL;
    }
}

int imask_sketch_apply(const imask_geometry* g, const imask_levels* lv, int32_t k, int32_t adjoint,
                       const void* work, const float* in, float* out, void* stream)
{
    if (!geometry_ok(g) || !work || !in || !out || in == out) return IMASK_EINVAL;
    const Layout L = make_layout(*g);
    if (!levels_ok(lv, L.lmax) || k < 0 || k >= lv->r) return IMASK_EINVAL;
    float* W = (float*)work;
    hipStream_t s = (hipStream_t)stream;
    if (!adjoint) {
        PrepArgs pa;
        FwdArgs fa{};
        forward_plan(L, *lv, k, in, W, pa, fa);
        fwd_common(L, W, fa);
        fa.mode = FWD_STORE;
        fa.out = out;
        IMK_TRY(launch_prep(pa, s));
        IMK_TRY(launch_fwd(fa, s));
        return IMASK_OK;
    }
    if (k > 0) {
        const int l = lv->log2f[k];
        return backproject_raw(L, W, l, in, out, 1.0f / (float)(1 << (2 * l)), 0, 1, s);
    }
    if (lv->r == 1) return backproject_raw(L, W, 0, in, out, 1.0f, 0, 1, s);
    if (lv->full_mode == IMASK_FULL_PAPER) {
        if (int rc = backproject_raw(L, W, 0, in, W + L.craw[0], 1.0f, 0, 0, s)) return rc;
        return imask_resample(g->n, 0, IMASK_COMPENSATE, lv, W + L.craw[0], out, stream);
    }
    if (int rc = backproject_raw(L, W, 0, in, out, (float)(1.0 / lv->p[0]), 0, 1, s)) return rc;
    for (int j = 1; j < lv->r; ++j) {
        const int l = lv->log2f[j];
        const float coef = (float)(-lv->p[j] / lv->p[0] / (double)(1 << (2 * l)));
        if (int rc = backproject_raw(L, W, l, in, out, coef, 1, 1, s)) return rc;
    }
    return IMASK_OK;
}

int imask_draws(const imask_params* prm, const imask_levels* lv, uint64_t k0, int32_t count, int32_t* out_host)
{
    if (!prm || !lv || !out_host || count < 0) return IMASK_EINVAL;
    if (!levels_ok(lv, IMASK_MAX_LOG2F)) return IMASK_EINVAL;
    uint64_t thr[IMASK_MAX_LEVELS];
    draw_thresholds(*lv, thr);
    for (int32_t q = 0; q < count; ++q) out_host[q] = draw_one(*prm, thr, k0 + (uint64_t)q);
    return IMASK_OK;
}

static int check_problem(const imask_geometry* g, const imask_levels* lv, const imask_reg* reg,
                         const imask_params* prm, const float* b, const imask_state* s)
{
    if (!geometry_ok(g)) return IMASK_EINVAL;
    const int lmax = level_limit(g->n);
    if (!levels_ok(lv, lmax) || !reg_ok(reg) || !prm || !b || !state_ok(s)) return IMASK_EINVAL;
    if (!(prm->sigma > 0.0) || !std::isfinite(prm->sigma)) return IMASK_EINVAL;
    return IMASK_OK;
}

int imask_step(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, const imask_reg* reg,
               const imask_params* prm, const float* const* b, imask_state* s, int32_t n_steps, void* stream)
{
    if (n_problems < 0 || n_steps < 0 || (n_problems > 0 && (!g || !lv || !reg || !prm || !b || !s)))
        return IMASK_EINVAL;
    for (int q = 0; q < n_problems; ++q)
        if (int rc = check_problem(g + q, lv + q, reg + q, prm + q, b[q], s + q)) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (int it = 0; it < n_steps; ++it)
        for (int q = 0; q < n_problems; ++q) {
            const Layout L = make_layout(g[q]);
            if (int rc = one_step(g[q], L, lv[q], reg[q], prm[q], b[q], s[q], st)) return rc;
        }
    return IMASK_OK;
}

int imask_solve(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, const imask_reg* reg,
                const imask_params* prm, const float* const* b, imask_state* s, double budget, int32_t budget_kind,
                void* stream)
{
    if (n_problems < 0 || !(budget >= 0.0) || !std::isfinite(budget) ||
        (budget_kind != IMASK_BUDGET_ITERS && budget_kind != IMASK_BUDGET_EPOCHS))
        return IMASK_EINVAL;
    if (n_problems > 0 && (!g || !lv || !reg || !prm || !b || !s)) return IMASK_EINVAL;
    for (int q = 0; q < n_problems; ++q)
        if (int rc = check_problem(g + q, lv + q, reg + q, prm + q, b[q], s + q)) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (int q = 0; q < n_problems; ++q) {
        const Layout L = make_layout(g[q]);
        const uint64_t k_start = s[q].k;
        const double e_start = s[q].epochs;
        for (;;) {
            const bool done = budget_kind == IMASK_BUDGET_ITERS ? (double)(s[q].k - k_start) >= budget
                                                                : s[q].epochs - e_start >= budget;
            if (done) break;
            if (int rc = one_step(g[q], L, lv[q], reg[q], prm[q], b[q], s[q], st)) return rc;
        }
    }
    return IMASK_OK;
}

}  // extern "C"
