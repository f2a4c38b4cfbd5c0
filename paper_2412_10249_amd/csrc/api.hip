// api.hip - the C ABI of libimask (include/imask.h): argument validation,
// workspace layout, the host-side sketch draw and the per-step launch
// sequence of Alg. 1.  All device work goes to the caller's stream; no call
// allocates or frees, and only set-up calls synchronise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "imask.h"
#include "internal.h"

namespace imk {

static size_t align64(size_t f) { return (f + 63) & ~(size_t)63; }

constexpr size_t kDotPartials = 256;                 // per-block partials of a dot product
constexpr size_t kConstDotDoubles = kDotPartials + 64;  // partials + result, keeps floats aligned

static int level_limit(int n)
{
    int l = 0;
    while (l < IMASK_MAX_LOG2F && (n % (2 << l)) == 0 && (n >> (l + 1)) >= 2) ++l;
    return l;
}

// A listed angle steps along rows when |cos| >= |sin| (FP64, host libm):
// the step between samples then stays within sqrt(2) pixels.
static bool listed_row(double th) { return std::fabs(std::cos(th)) >= std::fabs(std::sin(th)); }

// Row-stepping count of a listed angle set.  Launch sizes need it on every
// call, so the last sets seen by this thread are kept and recognised by value.
static int listed_nrow(const double* ang, int na)
{
    struct Seen {
        std::vector<double> a;
        int nrow = 0;
    };
    static thread_local Seen seen[4];
    static thread_local int next = 0;
    for (const Seen& e : seen)
        if ((int)e.a.size() == na && std::memcmp(e.a.data(), ang, sizeof(double) * na) == 0) return e.nrow;
    int nrow = 0;
    for (int a = 0; a < na; ++a) nrow += listed_row(ang[a]) ? 1 : 0;
    seen[next].a.assign(ang, ang + na);
    seen[next].nrow = nrow;
    next = (next + 1) & 3;
    return nrow;
}

static double extent_of(const imask_geometry& g) { return g.extent > 0 ? g.extent : 1.0; }
static bool is_fan(const imask_geometry& g) { return g.src_dist != 0.0; }
// Fan beam: the magnification from the centre onto the detector.
static double fan_mag(const imask_geometry& g) { return (g.src_dist + g.det_dist) / g.src_dist; }
static double spacing_of(const imask_geometry& g)
{
    if (g.det_spacing > 0) return g.det_spacing;
    const double h = 2.0 * extent_of(g) / g.n;
    return is_fan(g) ? h * fan_mag(g) : h;
}

Layout make_layout(const imask_geometry& g)
{
    Layout L;
    L.n = g.n;
    L.na = g.n_angles;
    L.nd = g.n_det;
    L.lmax = level_limit(g.n);
    L.E = extent_of(g);
    L.ds = spacing_of(g);
    L.s0 = g.det_offset;
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
    const size_t d = (size_t)g.n * g.n;
    L.part_floats = kPartImages * d;
    if (is_fan(g))
        L.part_floats = std::max(L.part_floats, std::min(kFanPartImages * d, kFanPartFloats));
    else
        L.part_floats = std::max(L.part_floats, std::min(kParPartImages * d, kParPartFloats));
    off = align64(off + L.part_floats);
    L.ptmp = off;
    off = align64(off + (size_t)g.n * g.n);
    const size_t m = (size_t)g.n_angles * g.n_det;
    for (int l = 0; l <= L.lmax; ++l) {
        // LDS bands of the level image for either beam (the fan forward
        // walks each ray's own line through the same bands)
        fwd_bands(side(g.n, l), g.n_angles, g.n_det, &L.fbands[l], &L.frows[l]);
        // sized for the default band layout; tuned shapes use no more bands
        int cap = L.fbands[l], rows_cap = 0;
        fwd_bands_default(side(g.n, l), g.n_angles, g.n_det, &cap, &rows_cap);
        L.fpart[l] = off;
        off = align64(off + (size_t)std::max(cap, L.fbands[l]) * m);
    }
    L.angtab = off;
    off = align64(off + 4 * (size_t)g.n_angles);
    L.flag = off;
    off = align64(off + 1);
    if (is_fan(g)) {
        L.fan = 1;
        L.D = g.src_dist;
        L.Dd = g.det_dist;
        // The transpose estimates bin coordinates in FP32: every point it
        // projects lies within 1.6E of the centre, so |t| <= (D + Dd) 1.6E /
        // (D - 1.6E) < 3.8 (D + Dd)/D E, and the estimate's error stays below
        // 32 ulp of the largest term of (t - s0)/ds + (n_det - 1)/2; the
        // margin is 1e-2 bin plus ten times that.
        const double big = 3.8 * fan_mag(g) * L.E / L.ds + std::fabs(g.det_offset) / L.ds + g.n_det;
        L.bmargin = 1e-2 + 10.0 * 32.0 * std::ldexp(1.0, -24) * big;
        L.fray = off;
        off = align64(off + m * (sizeof(FanRay) / sizeof(float)));
        L.fview = off;
        off = align64(off + (size_t)g.n_angles * (sizeof(FanView) / sizeof(float)));
        L.ftab = off;
        off = align64(off + m * (sizeof(FanTab) / sizeof(float)));
        // Adjacent bins of a flat detector subtend at least
        // ds L / (L^2 + t_max^2) radians at the source (L = D + Dd, t_max the
        // largest |t_b|), and every cell the transpose updates lies at least
        // D - 1.6E from the source: two rays b bins apart are at least
        // b times that far apart across a row or column there.
        const double Lsd = g.src_dist + g.det_dist;
        const double tmax = 0.5 * (g.n_det - 1) * L.ds + std::fabs(g.det_offset);
        L.min_sep = (g.src_dist - 1.6 * L.E) * L.ds * Lsd / (Lsd * Lsd + tmax * tmax);
        L.split = angle_split(g.n_angles);  // unused by the fan kernels
    } else if (g.angles) {
        L.listed = 1;
        L.split = AngleSplit{};
        L.split.nrow = listed_nrow(g.angles, g.n_angles);
        L.split.ncol = g.n_angles - L.split.nrow;
    } else {
        L.split = angle_split(g.n_angles);
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
    if (!std::isfinite(g->det_spacing) || !std::isfinite(g->det_offset) || !std::isfinite(g->extent)) return false;
    if (!std::isfinite(g->src_dist) || !std::isfinite(g->det_dist)) return false;
    // bounds that keep every fixed-point coordinate far inside what the FP32
    // range estimates resolve (the rows' zero padding absorbs their error)
    const double E = extent_of(*g);
    if (E < 1e-100 || E > 1e100) return false;
    double mag = 1.0;
    if (is_fan(*g)) {
        // the source stays outside every pixel's tap interval (all within
        // 2E of the centre), so each point projects onto the detector; the
        // upper bounds keep the fixed-point coordinates in range
        if (!(g->src_dist > 2 * E) || g->src_dist > 1e4 * E) return false;
        if (!(g->det_dist >= 0) || g->det_dist > 1e4 * E) return false;
        mag = fan_mag(*g);
    }
    const double h = 2.0 * E / g->n * mag;
    if (g->det_spacing > 0 && (g->det_spacing < h / 64 || g->det_spacing > 64 * h)) return false;
    if (std::fabs(g->det_offset) > 4 * E * mag) return false;
    if (g->angles)
        for (int a = 0; a < g->n_angles; ++a)
            if (!std::isfinite(g->angles[a])) return false;
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
    if (lv->n_blocks < 0 || lv->n_blocks > IMASK_MAX_BLOCKS) return false;
    return lv->full_mode == IMASK_FULL_PAPER || lv->full_mode == IMASK_FULL_UNBIASED;
}

static bool reg_ok(const imask_reg* r)
{
    if (!r || !(r->lambda > 0.0) || !std::isfinite(r->lambda)) return false;
    if (r->kind == IMASK_REG_TIKHONOV) return true;
    const bool inner = r->tv_inner >= 1 && r->tv_inner <= IMASK_MAX_TV_INNER;
    if (r->kind == IMASK_REG_TV) return r->tv_weight > 0.0 && std::isfinite(r->tv_weight) && inner;
    if (r->kind != IMASK_REG_SMOOTH_TV) return false;
    return r->tv_weight >= 0.0 && std::isfinite(r->tv_weight) && r->tv_eps > 0.0 && std::isfinite(r->tv_eps) && inner;
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

// Measurement block of draw k: the low word of the same output whose high
// word picks the sketch, scaled to the block count.
static int draw_block(const imask_params& prm, uint64_t k, int nblk)
{
    const uint64_t lo = mix_at(mix_at(prm.seed, prm.stream_id), k) & 0xffffffffULL;
    return (int)((lo * (uint64_t)nblk) >> 32);
}

static int block_count(const imask_levels& lv) { return lv.n_blocks > 1 ? lv.n_blocks : 1; }

// Angles [a0, a1) of measurement block j of nblk contiguous blocks.
static void block_angles(int na, int nblk, int j, int* a0, int* a1)
{
    *a0 = (int)(((long long)j * na) / nblk);
    *a1 = (int)(((long long)(j + 1) * na) / nblk);
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
    fa.fan = fan_at(L, W);
    fa.split = split_at(L, W);
    fa.n = L.n;
    fa.na = L.na;
    fa.nd = L.nd;
    fa.e0 = 0;
    fa.e1 = (long long)L.na * L.nd;
}

static BpArgs bp_args(const Layout& L, const float* W, int lvl, const float* y, float* out, float coef,
                      int accumulate, int prolong)
{
    BpArgs ba{};
    ba.consts = (const RayConst*)(W + L.consts);
    ba.fan = fan_at(L, W);
    ba.split = split_at(L, W);
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
    return ba;
}

static int backproject_raw(const Layout& L, const float* W, int lvl, const float* y, float* out, float coef,
                           int accumulate, int prolong, hipStream_t s)
{
    IMK_TRY(launch_bp(bp_args(L, W, lvl, y, out, coef, accumulate, prolong), s));
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

// FISTA extrapolation weights (t_j - 1) / t_{j+1}, t_0 = 1 (Beck-Teboulle).
static void fista_betas(int J, float* beta)
{
    double t = 1.0;
    for (int it = 0; it < J; ++it) {
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        beta[it] = (float)((t - 1.0) / tn);
        t = tn;
    }
}

// Whether a step of this problem is described by launch records (and can
// run batched): parallel beam, Alg. 1's parallel schedule with common draws,
// no measurement blocks, the standard tables.
static bool step_is_plain(const imask_geometry& g, const imask_levels& lv, const imask_params& prm,
                          const imask_state& st)
{
    return !is_fan(g) && prm.schedule == IMASK_SCHEDULE_PARALLEL && prm.draw_mode == IMASK_DRAW_COMMON &&
           block_count(lv) == 1 && !st.ztab;
}

// The launches of steps a2-a7 of one plain step for sketch k from the
// state's parity st.cur: restriction, forward projection and dual step,
// transposes, prolongation and primal step (the TV proxes follow it).
// Transposes of the UNBIASED full-resolution sketch take successive rounds:
// they share the workspace's partial images.
static void step_records(const imask_geometry& g, const Layout& L, const imask_levels& lv, const imask_reg& reg,
                         const imask_params& prm, const float* bdat, const imask_state& st, int k, Launches& out,
                         bool fuse, bool skip_prep = false)
{
    // the UNBIASED full-resolution sketch applies every level: with `fuse`
    // its forward terms share one launch and its coarse transposes one per
    // tile shape (the batched path runs a variant's launches together anyway)
    const bool multi = fuse && k == 0 && lv.r > 1 && lv.full_mode == IMASK_FULL_UNBIASED;
    float* W = (float*)st.work;
    const int cur = st.cur, nxt = 1 - cur;
    const int lmax_set = lv.log2f[lv.r - 1];
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
    if (!skip_prep) plan_prep(pa, out);
    if (multi)
        plan_fwd_fused(fa, out);
    else
        plan_fwd(fa, out);

    const double tau = prm.sigma / reg.lambda;
    const bool tv = reg.kind != IMASK_REG_TIKHONOV;
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
        pr.pavg[j] = (float)lv.p[j];
        pr.craw[j] = W + L.craw[lv.log2f[j]];
    }
    pr.phi = st.phi;
    phi_offsets(g, lv, pr.phi_off);
    pr.nblk = 1;
    pr.jblk = 0;
    pr.blk_stride = 0;
    for (int j = 0; j < lv.r; ++j) pr.blk_stride += (long long)(g.n >> lv.log2f[j]) * (g.n >> lv.log2f[j]);
    pr.x_old = st.x[cur];
    pr.x_out = tv ? W + L.vbuf : st.x[nxt];
    pr.tau = (float)tau;
    pr.prox_scale = tv ? 1.0f : (float)(1.0 / (1.0 + tau * reg.lambda));
    pr.xbar = nullptr;
    pr.theta = (float)prm.theta;
    auto raw_bp = [&](int l) { return bp_args(L, W, l, st.y[cur], W + L.craw[l], 1.0f, 0, 0); };
    if (k > 0 || lv.r == 1) {
        plan_bp_primal(raw_bp(lv.log2f[k]), pr, out);
    } else if (lv.full_mode == IMASK_FULL_PAPER && sum_primal_tile_fits(pr)) {
        // level 0's partial images summed per tile inside the primal step
        BpOwnArgs used;
        plan_bp_main(raw_bp(0), 0, out, &used);
        plan_sum_primal_tile(used, pr, out);
    } else {
        plan_bp(raw_bp(0), 0, out);
        if (lv.full_mode == IMASK_FULL_UNBIASED) {
            BpArgs coarse[IMASK_MAX_LEVELS];
            for (int j = 1; j < lv.r; ++j) coarse[j - 1] = raw_bp(lv.log2f[j]);
            // after level 0's ordered sum the whole partial-image buffer is
            // free for the coarse levels side by side: one launch per
            // direction when fused (the single-problem path), the same
            // launches one by one in the batched path
            plan_bp_coarse(coarse, lv.r - 1, L.part_floats, multi, 1, out);
        }
        plan_primal(pr, out);
    }
}

// The forward's restriction can be carried from one step to the next: a
// step whose prox writes it for the next step's sketch sets `made`, and the
// next step of the same call, given `ready`, launches no k_prep.  `more`
// says whether another step of this problem follows in the call (when not,
// nothing is carried).
struct PrepCarry {
    bool ready = false;
    bool made = false;
};

// The forward sketch (dual draw) of step k.
static int fwd_sketch(const imask_params& prm, const uint64_t* thr, uint64_t k)
{
    if (prm.draw_mode != IMASK_DRAW_INDEPENDENT) return draw_one(prm, thr, k);
    imask_params dual = prm;
    dual.stream_id = prm.dual_stream_id;
    return draw_one(dual, thr, k);
}

static int one_step(const imask_geometry& g, const Layout& L, const imask_levels& lv, const imask_reg& reg,
                    const imask_params& prm, const float* bdat, imask_state& st, hipStream_t s,
                    PrepCarry* carry = nullptr, bool more = false)
{
    const bool prep_ready = carry && carry->ready;
    if (carry) carry->made = false;
    uint64_t thr[IMASK_MAX_LEVELS];
    draw_thresholds(lv, thr);
    const int k = draw_one(prm, thr, st.k);  // primal sketch (K_k^T, phi)
    int kd = k;                                // dual sketch (K_kd, psi)
    if (prm.draw_mode == IMASK_DRAW_INDEPENDENT) {
        imask_params dual = prm;
        dual.stream_id = prm.dual_stream_id;
        kd = draw_one(dual, thr, st.k);
    }
    float* W = (float*)st.work;
    const int cur = st.cur, nxt = 1 - cur;
    const int lmax_set = lv.log2f[lv.r - 1];
    const bool plain = step_is_plain(g, lv, prm, st);
    // Alg. 1 takes both steps from (x^k, y^k); ImaSk-Seq (Sec. 5) projects the
    // extrapolated point and backprojects the new dual iterate
    const bool seq = prm.schedule == IMASK_SCHEDULE_SEQUENTIAL;
    const float* x_fwd = seq ? st.xbar : st.x[cur];
    const float* y_bp = seq ? st.y[nxt] : st.y[cur];
    // measurement blocks (Sec. 6 outlook): this step's sketch is
    // K_kb = S E_b K_k on the rows of angle block b, drawn uniformly
    const int nblk = block_count(lv);
    const int jb = nblk > 1 ? draw_block(prm, st.k, nblk) : 0;
    int a0 = 0, a1 = g.n_angles;
    if (nblk > 1) block_angles(g.n_angles, nblk, jb, &a0, &a1);
    const AngleSplit blk_split = angle_split_range(g.n_angles, a0, a1);
    const float blk_coef = (float)nblk;

    // a2-a4: restriction, forward projection, dual SAGA step and psi refresh
    PrepArgs pa;
    FwdArgs fa{};
    forward_plan(L, lv, kd, x_fwd, W, pa, fa);
    fwd_common(L, W, fa);
    if (st.ztab) {  // compact dual tables (Remark 1): project x - z_k, refresh z_k
        long long zoff[IMASK_MAX_LEVELS];
        phi_offsets(g, lv, zoff);
        pa.snap = st.ztab + zoff[kd];
        pa.snap_lvl = lv.log2f[kd];
        fa.compact = 1;
    }
    fa.mode = FWD_DUAL;
    fa.y_old = st.y[cur];
    fa.y_new = st.y[nxt];
    fa.bdat = bdat;
    fa.psi = st.psi;
    fa.r = lv.r;
    fa.kidx = kd;
    for (int j = 0; j < lv.r; ++j) fa.p[j] = (float)(lv.p[j] / nblk);
    if (nblk > 1) {
        for (int t = 0; t < fa.nterms; ++t) fa.term[t].coef *= blk_coef;
        fa.split = blk_split;
        fa.fan.va = a0;
        fa.fan.vb = a1;
        fa.e0 = (long long)a0 * g.n_det;
        fa.e1 = (long long)a1 * g.n_det;
    }
    fa.sigma = (float)prm.sigma;
    fa.inv1ps = (float)(1.0 / (1.0 + prm.sigma));
    if (plain) {
        // the same launches the batched path stores
        Launches recs;
        step_records(g, L, lv, reg, prm, bdat, st, k, recs, true, prep_ready);
        // the parallel schedule: the transpose reads y^k, so the forward
        // half's last launch can share the transpose's
        merge_reduce_into_transpose(recs);
        merge_forward_into_transpose(recs);
        IMK_TRY(launch_records(recs, s));
    } else {
        if (!prep_ready) IMK_TRY(launch_prep(pa, s));
        IMK_TRY(launch_fwd(fa, s));
    }

    // a6-a7: prolongation / compensation, primal SAGA step, phi refresh
    const double tau = prm.sigma / reg.lambda;
    const bool tv = reg.kind != IMASK_REG_TIKHONOV;  // the prox runs in its own kernel
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
        pr.pavg[j] = (float)(lv.p[j] / nblk);
        pr.craw[j] = W + L.craw[lv.log2f[j]];
    }
    pr.phi = st.phi;
    phi_offsets(g, lv, pr.phi_off);
    pr.nblk = nblk;
    pr.jblk = jb;
    pr.blk_stride = 0;
    for (int j = 0; j < lv.r; ++j) pr.blk_stride += (long long)(g.n >> lv.log2f[j]) * (g.n >> lv.log2f[j]);
    pr.x_old = st.x[cur];
    pr.x_out = tv ? W + L.vbuf : st.x[nxt];
    pr.tau = (float)tau;
    pr.prox_scale = tv ? 1.0f : (float)(1.0 / (1.0 + tau * reg.lambda));
    // extrapolation xbar^{k+1} = x^{k+1} + theta (x^{k+1} - x^k), fused into
    // whichever kernel writes x^{k+1}
    pr.xbar = seq && !tv ? st.xbar : nullptr;
    pr.theta = (float)prm.theta;
    // a5: raw backprojections R_l^T y needed by sketch k.  A sketch that
    // needs one (coarse, or the only level) takes the primal step in the
    // epilogue of that backprojection's ordered sum.
    auto raw_bp = [&](int l) {  // R_l^T y (times S on the block's rows only)
        BpArgs ba = bp_args(L, W, l, y_bp, W + L.craw[l], blk_coef, 0, 0);
        if (nblk > 1) {
            ba.split = blk_split;
            ba.fan.va = a0;
            ba.fan.vb = a1;
        }
        return ba;
    };
    if (plain) {
        // launched with the forward records above
    } else if (k > 0 || lv.r == 1) {
        IMK_TRY(launch_bp_primal(raw_bp(lv.log2f[k]), pr, s));
    } else if (lv.full_mode == IMASK_FULL_PAPER && sum_primal_tile_fits(pr)) {
        // level 0's partial images summed per tile inside the primal step,
        // as on the plain path
        BpOwnArgs used;
        IMK_TRY(launch_bp_main(raw_bp(0), s, used));
        Launches r;
        plan_sum_primal_tile(used, pr, r);
        IMK_TRY(launch_records(r, s));
    } else {
        IMK_TRY(launch_bp(raw_bp(0), s));
        if (lv.full_mode == IMASK_FULL_UNBIASED)
            for (int j = 1; j < lv.r; ++j) IMK_TRY(launch_bp(raw_bp(lv.log2f[j]), s));
        IMK_TRY(launch_primal(pr, s));
    }

    // a8: the paper's TV prior: dual FGP from the kept dual pair at
    // v / (1 + tau lam) with weight tau w / (1 + tau lam)
    if (reg.kind == IMASK_REG_TV) {
        const double sc = 1.0 + tau * reg.lambda;
        TvdArgs ta{};
        ta.n = g.n;
        ta.J = reg.tv_inner;
        ta.v = W + L.vbuf;
        ta.pin = st.tvd[cur];
        ta.pout = st.tvd[nxt];
        ta.out = st.x[nxt];
        ta.u0 = st.x[cur];
        ta.xbar = seq ? st.xbar : nullptr;
        ta.theta = (float)prm.theta;
        ta.inv_scale = (float)(1.0 / sc);
        ta.gamma = (float)(tau * reg.tv_weight / sc);
        ta.inv8g = (float)(1.0 / (8.0 * tau * reg.tv_weight / sc));
        fista_betas(reg.tv_inner, ta.beta);
        IMK_TRY(launch_tvd(ta, s));
    }
    // a8: smoothed-TV prox by FISTA, warm-started at x^k
    if (reg.kind == IMASK_REG_SMOOTH_TV) {
        TvArgs ta{};
        ta.n = g.n;
        ta.J = reg.tv_inner;
        ta.v = W + L.vbuf;
        ta.u0 = st.x[cur];
        ta.out = st.x[nxt];
        ta.xbar = seq ? st.xbar : nullptr;
        ta.theta = (float)prm.theta;
        ta.tau_w = (float)(tau * reg.tv_weight);
        ta.tau_lam = (float)(tau * reg.lambda);
        ta.eps = (float)reg.tv_eps;
        ta.invL = (float)(1.0 / (1.0 + tau * reg.lambda + 8.0 * tau * reg.tv_weight / reg.tv_eps));
        fista_betas(reg.tv_inner, ta.beta);
        // the next step's restriction of x^{k+1} (the plain schedule projects
        // x itself; compact tables restrict against a snapshot, so they keep
        // k_prep)
        if (carry && more && !seq && !st.ztab) {
            FwdArgs fn{};
            forward_plan(L, lv, fwd_sketch(prm, thr, st.k + 1), st.x[nxt], W, ta.next, fn);
            if (tv_prep_fusable(g.n, ta.next)) {
                ta.prep_next = 1;
                carry->made = true;
            }
        }
        IMK_TRY(launch_tv(ta, s));
    }

    if (carry) carry->ready = carry->made;
    st.cur = nxt;
    st.k += 1;
    if (nblk > 1)
        st.epochs += sketch_cost(lv, k) * (double)(a1 - a0) / g.n_angles;
    else
        st.epochs += kd == k ? sketch_cost(lv, k) : 0.5 * (sketch_cost(lv, k) + sketch_cost(lv, kd));
    return IMASK_OK;
}

// ---- batched steps ----

constexpr int kMaxBatch = 4096;

struct BatchLayout {
    size_t prob = 0, rec = 0, nrec = 0, items = 0, off = 0, sel = 0, nsegs = 0, segc = 0, seg_off = 0, seg = 0,
           rank = 0, blobs = 0, total = 0;  // bytes
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static BatchLayout batch_layout(int n, int r_max, size_t nblobs)
{
    BatchLayout B;
    size_t o = 0;
    B.prob = o;
    o = align256(o + (size_t)n * sizeof(BatchProb));
    B.rec = o;
    o = align256(o + (size_t)n * r_max * 2 * kMaxRec * sizeof(BatchRec));
    B.nrec = o;
    o = align256(o + (size_t)n * r_max * 2 * sizeof(int));
    B.items = o;
    o = align256(o + (size_t)n * r_max * 2 * kNumVariants * kRounds * sizeof(int));
    B.off = o;
    o = align256(o + (size_t)kNumVariants * kRounds * (n + 1) * sizeof(int));
    B.sel = o;
    o = align256(o + (size_t)n * sizeof(int));
    B.nsegs = o;
    o = align256(o + (size_t)n * r_max * 2 * kNumVariants * kRounds * sizeof(int));
    B.segc = o;
    o = align256(o + (size_t)kNumVariants * kRounds * (n + 1) * sizeof(int));
    B.seg_off = o;
    o = align256(o + (size_t)(kNumVariants * kRounds + 1) * sizeof(int));
    B.seg = o;
    o = align256(o + (size_t)n * kMaxRec * 2 * sizeof(int));
    B.rank = o;
    o = align256(o + (size_t)n * sizeof(int));
    B.blobs = o;
    o = align256(o + nblobs * kBlobBytes);
    B.total = o;
    return B;
}

static BatchView batch_view(void* batch, int n, int r_max)
{
    const BatchLayout B = batch_layout(n, r_max, 0);
    unsigned char* base = (unsigned char*)batch;
    BatchView v;
    v.n = n;
    v.r_max = r_max;
    v.prob = (BatchProb*)(base + B.prob);
    v.rec = (const BatchRec*)(base + B.rec);
    v.nrec = (const int*)(base + B.nrec);
    v.items = (const int*)(base + B.items);
    v.blobs = base + B.blobs;
    v.off = (int*)(base + B.off);
    v.sel = (int*)(base + B.sel);
    v.nsegs = (const int*)(base + B.nsegs);
    v.segc = (int*)(base + B.segc);
    v.seg_off = (int*)(base + B.seg_off);
    v.seg = (int*)(base + B.seg);
    v.rank = (const int*)(base + B.rank);
    return v;
}

// A batched problem: parallel beam, Alg. 1's parallel schedule with common
// draws, no measurement blocks, standard tables, the Tikhonov prior.
static int batch_check(int n, const imask_geometry* g, const imask_levels* lv)
{
    if (n < 1 || n > kMaxBatch || !g || !lv) return IMASK_EINVAL;
    for (int q = 0; q < n; ++q) {
        if (!geometry_ok(g + q) || !levels_ok(lv + q, level_limit(g[q].n))) return IMASK_EINVAL;
        if (is_fan(g[q]) || lv[q].n_blocks > 1) return IMASK_ENOTSUP;
    }
    return IMASK_OK;
}

static int batch_rmax(int n, const imask_levels* lv)
{
    int r = 1;
    for (int q = 0; q < n; ++q) r = std::max(r, (int)lv[q].r);
    return r;
}

// The records of sketch k of problem q with placeholder buffers: the launch
// shapes (grids, LDS) depend on the geometry and level set only.
static void shape_records(const imask_geometry& g, const imask_levels& lv, int k, Launches& out)
{
    const Layout L = make_layout(g);
    imask_state st{};
    float* fake = (float*)(uintptr_t)4096;
    st.x[0] = st.x[1] = st.y[0] = st.y[1] = st.phi = st.psi = fake;
    st.work = fake;
    imask_reg reg{IMASK_REG_TIKHONOV, 1.0, 0.0, 1.0, 1};
    imask_params prm{};
    prm.sigma = 1.0;
    step_records(g, L, lv, reg, prm, fake, st, k, out, false);
}

// The stage slot of a launch: its round and LDS class.
static int stage_slot(const Launch& L) { return L.round * kLdsClasses + lds_class(L.lds); }

// Per (variant, round): the largest dynamic LDS and the sum over problems of
// their largest item count, from the shapes alone.  The two reduce variants
// differ only in the alignment of the caller's buffers, so both are sized
// alike.
struct StageShape {
    int lds[kNumVariants][kRounds];
    long long ub[kNumVariants][kRounds];
    int rounds;
};

static void batch_shapes(int n, const imask_geometry* g, const imask_levels* lv, StageShape& sh, size_t* nblobs)
{
    std::memset(&sh, 0, sizeof(sh));
    sh.rounds = 1;
    size_t blobs = 0;
    for (int q = 0; q < n; ++q) {
        long long best[kNumVariants][kRounds] = {};
        for (int k = 0; k < lv[q].r; ++k) {
            Launches recs;
            shape_records(g[q], lv[q], k, recs);
            blobs += 2 * recs.size();
            long long it[kNumVariants][kRounds] = {};
            for (const Launch& L : recs) {
                const int slot = stage_slot(L);
                it[L.variant][slot] += (long long)L.gx * L.gy * L.gz;
                sh.lds[L.variant][slot] = std::max(sh.lds[L.variant][slot], L.lds);
                sh.rounds = std::max(sh.rounds, L.round + 1);
            }
            for (int v = 0; v < kNumVariants; ++v)
                for (int j = 0; j < kRounds; ++j) best[v][j] = std::max(best[v][j], it[v][j]);
        }
        for (int j = 0; j < kRounds; ++j) {
            const long long red = std::max(best[V_RED4][j], best[V_RED1][j]);
            best[V_RED4][j] = best[V_RED1][j] = red;
        }
        for (int v = 0; v < kNumVariants; ++v)
            for (int j = 0; j < kRounds; ++j) sh.ub[v][j] += best[v][j];
    }
    if (nblobs) *nblobs = blobs;
}

// Where a variant runs in a batched step: 0 restriction, forward and dual
// step; in each round 1 the transposes, then 2 their ordered sums; 3 the
// fused sums with the primal step and the primal step.
static int variant_phase(int v)
{
    switch (v) {
    case V_PREP: case V_FWD_BAND: case V_FWD_DIRECT: case V_RED4: case V_RED1: return 0;
    case V_BP28: case V_BP44: case V_BP14: case V_BP12: case V_BP24: return 1;
    case V_SUM4: case V_SUM1: return 2;
    case V_SUMP4: case V_SUMP1: case V_PRIMAL: case V_SUMPT: return 3;
    default: return -1;
    }
}

// Resident workgroups of a batched variant per CU (LDS and threads).
static int batch_wgs_per_cu(int v, int lds)
{
    const size_t need = (size_t)lds + variant_static_lds(v);
    const int by_lds = (int)std::max<size_t>(1, (size_t)(160 * 1024) / std::max<size_t>(need, 1));
    const int by_threads = std::max(1, 2048 / variant_threads(v));
    return std::max(1, std::min(by_lds, by_threads));
}

// ---- the workspace-free transpose (imask_backproject_noalloc) ----

// Device memory of imask_backproject_noalloc: one copy per GPU, held until
// the process ends.  Host code never passes this name to a kernel (on the
// host it is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[IMASK_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// The array's address on the current device, looked up once per device.
static int scratch_of_current_device(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return IMASK_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return IMASK_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return IMASK_OK;
}

// The part of a workspace the transpose reads and writes, packed from offset
// 0: projector constants of every level, the partial images (as many as the
// workspace holds, so the launches are those of imask_backproject), the
// coarse result before prolongation.
static Layout transpose_layout(const imask_geometry& g)
{
    Layout L = make_layout(g);
    size_t off = 0;
    L.consts = off;
    off = align64(off + (size_t)(L.lmax + 1) * g.n_angles * kConstStride);
    L.part = off;
    off = align64(off + L.part_floats);
    L.ptmp = off;
    off = align64(off + (size_t)g.n * g.n);
    L.total = off;
    return L;
}

}  // namespace imk

using namespace imk;

static int check_problem(const imask_geometry* g, const imask_levels* lv, const imask_reg* reg,
                         const imask_params* prm, const float* b, const imask_state* s);


extern "C" {

size_t imask_workspace_bytes(const imask_geometry* g)
{
    if (!geometry_ok(g)) return 0;
    return make_layout(*g).total * sizeof(float);
}

size_t imask_phi_floats(const imask_geometry* g, const imask_levels* lv)
{
    if (!geometry_ok(g) || !levels_ok(lv, level_limit(g->n)) || lv->n_blocks > g->n_angles) return 0;
    size_t t = 0;
    for (int k = 0; k < lv->r; ++k) {
        const size_t nl = (size_t)(g->n >> lv->log2f[k]);
        t += nl * nl;
    }
    return t * (size_t)block_count(*lv);
}

int imask_block_draws(const imask_params* prm, const imask_levels* lv, uint64_t k0, int32_t count, int32_t* out_host)
{
    if (!prm || !lv || !out_host || count < 0) return IMASK_EINVAL;
    if (!levels_ok(lv, IMASK_MAX_LOG2F)) return IMASK_EINVAL;
    const int nblk = block_count(*lv);
    for (int32_t q = 0; q < count; ++q) out_host[q] = nblk > 1 ? draw_block(*prm, k0 + (uint64_t)q, nblk) : 0;
    return IMASK_OK;
}

// Fan-beam lines in FP64 (host libm): view a's source D (cos b, sin b), its
// bin b's detector point -Dd (cos b, sin b) + t_b (-sin b, cos b), the ray's
// unit normal (ct, st) = (-dy, dx)/|d| for d = detector point - source, and
// s = (ct, st) . source; then the row-stepping form of FanRay.
static void fan_tables(const imask_geometry& g, double ds, std::vector<FanRay>& rays, std::vector<FanView>& views)
{
    const int na = g.n_angles, nd = g.n_det;
    const double D = g.src_dist, Dd = g.det_dist;
    rays.assign((size_t)na * nd, FanRay{});
    views.assign(na, FanView{});
    for (int a = 0; a < na; ++a) {
        const double beta = g.angles ? g.angles[a] : 2.0 * M_PI * a / na;
        const double cb = std::cos(beta), sb = std::sin(beta);
        FanView& v = views[a];
        v.c = cb;
        v.s = sb;
        const double srcx = D * cb, srcy = D * sb;
        for (int b = 0; b < nd; ++b) {
            const double t = (b - (nd - 1) / 2.0) * ds + g.det_offset;
            const double detx = -Dd * cb + t * -sb, dety = -Dd * sb + t * cb;
            const double dx = detx - srcx, dy = dety - srcy;
            const double len = std::sqrt(dx * dx + dy * dy);
            const double ct = -dy / len, st = dx / len;
            const double sl = ct * srcx + st * srcy;
            FanRay& r = rays[(size_t)a * nd + b];
            r.row = std::fabs(ct) >= std::fabs(st) ? 1 : 0;
            const double c = r.row ? ct : st, o = r.row ? st : ct;
            r.P = sl / c;
            r.T = o / c;
            r.sec = 1.0 / std::fabs(c);
            v.has_row |= r.row;
            v.has_col |= 1 - r.row;
        }
    }
}

int imask_prepare(const imask_geometry* g, void* work, size_t work_bytes, void* stream)
{
    if (!geometry_ok(g) || !work) return IMASK_EINVAL;
    const Layout L = make_layout(*g);
    if (work_bytes < L.total * sizeof(float)) return IMASK_ESIZE;
    hipStream_t s = (hipStream_t)stream;
    IMK_TRY(launch_fill((float*)work, L.total, 0.0f, s));
    if (L.listed) {
        // angle table: radians, then perm (row-stepping indices, then
        // column-stepping ones, each ascending), then the row flags
        const int na = g->n_angles;
        std::vector<double> tab(2 * (size_t)na);
        std::memcpy(tab.data(), g->angles, sizeof(double) * na);
        int* perm = (int*)(tab.data() + na);
        int* rows = perm + na;
        int r = 0, c = L.split.nrow;
        for (int a = 0; a < na; ++a) {
            rows[a] = listed_row(g->angles[a]) ? 1 : 0;
            perm[rows[a] ? r++ : c++] = a;
        }
        if (r != L.split.nrow || c != na) return IMASK_EINVAL;
        if (hipMemcpyAsync((float*)work + L.angtab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)  // tab is freed on return
            return IMASK_EHIP;
    }
    if (L.fan) {
        std::vector<FanRay> rays;
        std::vector<FanView> views;
        fan_tables(*g, L.ds, rays, views);
        if (hipMemcpyAsync((float*)work + L.fray, rays.data(), sizeof(FanRay) * rays.size(), hipMemcpyHostToDevice,
                           s) != hipSuccess ||
            hipMemcpyAsync((float*)work + L.fview, views.data(), sizeof(FanView) * views.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)  // the tables are freed on return
            return IMASK_EHIP;
        return IMASK_OK;
    }
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

int imask_backproject_noalloc(const imask_geometry* g, int32_t log2f, const float* sino, float* x_full,
                              void* stream)
{
    if (!geometry_ok(g) || !sino || !x_full) return IMASK_EINVAL;
    if (g->angles || is_fan(*g)) return IMASK_ENOTSUP;
    const Layout L = transpose_layout(*g);
    if (log2f < 0 || log2f > L.lmax) return IMASK_EINVAL;
    if (L.total * sizeof(float) > (size_t)IMASK_NOALLOC_SCRATCH_BYTES) return IMASK_ESIZE;
    void* ptr = nullptr;
    if (int rc = scratch_of_current_device(&ptr)) return rc;
    float* W = (float*)ptr;
    hipStream_t s = (hipStream_t)stream;
    // every cell the transpose reads is written earlier in this call (the
    // constants, each partial image in full, the coarse result), so the
    // array's previous contents never matter and nothing is cleared
    IMK_TRY(launch_consts(*g, L, W, s));
    return backproject_raw(L, W, log2f, sino, x_full, 1.0f / (float)(1 << (2 * log2f)), 0, 1, s);
}

int imask_set_tiles(int32_t nl, int32_t n_angles, int32_t n_det, const imask_tiles* t)
{
    if (nl < 1 || nl > 16384 || n_angles < 1 || n_angles > 65536 || n_det < 1 || n_det > 8192) return IMASK_EINVAL;
    if (!t) {
        set_tiles(nl, n_angles, n_det, nullptr);
        return IMASK_OK;
    }
    Tiles tt;
    tt.bp_rows = t->bp_rows;
    tt.bp_waves = t->bp_waves;
    tt.bp_wg = t->bp_wg;
    tt.fwd_lds_kb = t->fwd_lds_kb;
    return set_tiles(nl, n_angles, n_det, &tt) ? IMASK_OK : IMASK_EINVAL;
}

int imask_get_tiles(int32_t nl, int32_t n_angles, int32_t n_det, imask_tiles* out)
{
    if (!out) return IMASK_EINVAL;
    const Tiles t = tiles_for(nl, n_angles, n_det);
    out->bp_rows = t.bp_rows;
    out->bp_waves = t.bp_waves;
    out->bp_wg = t.bp_wg;
    out->fwd_lds_kb = t.fwd_lds_kb;
    return IMASK_OK;
}

size_t imask_batch_bytes(int32_t n_problems, const imask_geometry* g, const imask_levels* lv)
{
    if (batch_check(n_problems, g, lv) != IMASK_OK) return 0;
    StageShape sh;
    size_t nblobs = 0;
    batch_shapes(n_problems, g, lv, sh, &nblobs);
    return batch_layout(n_problems, batch_rmax(n_problems, lv), nblobs).total;
}

int imask_batch_prepare(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, const imask_reg* reg,
                        const imask_params* prm, const float* const* b, const imask_state* s, double budget,
                        int32_t budget_kind, void* batch, size_t batch_bytes, int64_t* steps_out, void* stream)
{
    if (int rc = batch_check(n_problems, g, lv)) return rc;
    if (!reg || !prm || !b || !s || !batch || !(budget >= 0.0) || !std::isfinite(budget) ||
        (budget_kind != IMASK_BUDGET_ITERS && budget_kind != IMASK_BUDGET_EPOCHS))
        return IMASK_EINVAL;
    for (int q = 0; q < n_problems; ++q) {
        if (int rc = check_problem(g + q, lv + q, reg + q, prm + q, b[q], s + q)) return rc;
        if (!step_is_plain(g[q], lv[q], prm[q], s[q]) || reg[q].kind != IMASK_REG_TIKHONOV) return IMASK_ENOTSUP;
    }
    const int n = n_problems, r_max = batch_rmax(n, lv);
    StageShape sh;
    size_t nblobs = 0;
    batch_shapes(n, g, lv, sh, &nblobs);
    const BatchLayout B = batch_layout(n, r_max, nblobs);
    if (batch_bytes < B.total) return IMASK_ESIZE;
    for (int v = 0; v < kNumVariants; ++v)
        for (int j = 0; j < kRounds; ++j)
            if (sh.ub[v][j] > 0 && (size_t)sh.lds[v][j] + variant_static_lds(v) > 160 * 1024) return IMASK_ENOTSUP;
    std::vector<unsigned char> img(B.total, 0);
    BatchProb* probs = (BatchProb*)(img.data() + B.prob);
    BatchRec* recs = (BatchRec*)(img.data() + B.rec);
    int* nrec = (int*)(img.data() + B.nrec);
    int* items = (int*)(img.data() + B.items);
    int* nsegs = (int*)(img.data() + B.nsegs);
    // work order: the problems with the most samples per step first
    {
        std::vector<std::pair<double, int>> work(n);
        for (int q = 0; q < n; ++q) work[q] = {-(double)g[q].n * g[q].n_angles * g[q].n_det, q};
        std::stable_sort(work.begin(), work.end());
        int* rank = (int*)(img.data() + B.rank);
        for (int i = 0; i < n; ++i) rank[work[i].second] = i;
    }
    unsigned char* blobs = img.data() + B.blobs;
    int64_t steps = 0;
    size_t blob = 0;
    for (int q = 0; q < n; ++q) {
        const Layout L = make_layout(g[q]);
        BatchProb& pb = probs[q];
        uint64_t thr[IMASK_MAX_LEVELS];
        draw_thresholds(lv[q], thr);
        pb.stream_state = mix_at(prm[q].seed, prm[q].stream_id);
        pb.k = s[q].k;
        pb.epochs = s[q].epochs;
        pb.cur = s[q].cur;
        pb.r = lv[q].r;
        for (int j = 0; j < lv[q].r; ++j) {
            pb.thr[j] = thr[j];
            pb.cost[j] = sketch_cost(lv[q], j);
        }
        // the problem's last draw: the budget evaluated from the host draws
        uint64_t kk = s[q].k;
        if (budget_kind == IMASK_BUDGET_ITERS) {
            kk += (uint64_t)budget;
        } else {
            double e = 0.0;
            while (e < budget) e += sketch_cost(lv[q], draw_one(prm[q], thr, kk++));
        }
        pb.k_stop = kk;
        steps = std::max<int64_t>(steps, (int64_t)(kk - s[q].k));
        for (int k = 0; k < lv[q].r; ++k)
            for (int c = 0; c < 2; ++c) {
                imask_state st = s[q];
                st.cur = c;
                Launches rl;
                step_records(g[q], L, lv[q], reg[q], prm[q], b[q], st, k, rl, false);
                if ((int)rl.size() > kMaxRec) return IMASK_ENOTSUP;
                for (const Launch& La : rl)
                    if (La.variant >= kNumVariants || variant_phase(La.variant) < 0 || stage_slot(La) >= kRounds)
                        return IMASK_ENOTSUP;
                const size_t slot = ((size_t)q * r_max + k) * 2 + c;
                nrec[slot] = (int)rl.size();
                for (size_t t = 0; t < rl.size(); ++t) {
                    const Launch& La = rl[t];
                    BatchRec& R = recs[slot * kMaxRec + t];
                    R.variant = La.variant;
                    R.round = stage_slot(La);
                    R.blob = (int)blob;
                    R.gx = (int)La.gx;
                    R.gy = (int)La.gy;
                    R.gz = (int)La.gz;
                    R.items = (int)(La.gx * La.gy * La.gz);
                    R.lds = La.lds;
                    std::memcpy(blobs + blob * kBlobBytes, La.args, kBlobBytes);
                    ++blob;
                    int& it = items[(slot * kNumVariants + La.variant) * kRounds + R.round];
                    int& ns = nsegs[(slot * kNumVariants + La.variant) * kRounds + R.round];
                    R.ord = ns;
                    R.ibefore = it;
                    it += R.items;
                    ns += 1;
                }
            }
    }
    if (blob > nblobs) return IMASK_ESIZE;
    hipStream_t st = (hipStream_t)stream;
    for (int v = 0; v < kNumVariants; ++v)
        for (int j = 0; j < sh.rounds; ++j)
            if (sh.ub[v][j] > 0) IMK_TRY(batch_allow_lds(v, sh.lds[v][j]));
    if (hipMemcpyAsync(batch, img.data(), B.total, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)  // img is freed on return
        return IMASK_EHIP;
    if (steps_out) *steps_out = steps;
    return IMASK_OK;
}

// One part of a batched step (see imask_batch_step_part), with the stage
// shapes of these problems.
static int batch_part(int n, const imask_levels* lv, void* batch, int part, const StageShape& sh, hipStream_t s);

int imask_batch_step_part(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, void* batch,
                          int32_t part, void* stream)
{
    if (int rc = batch_check(n_problems, g, lv)) return rc;
    if (!batch || part < IMASK_BATCH_PLAN || part > IMASK_BATCH_ADVANCE) return IMASK_EINVAL;
    StageShape sh;
    batch_shapes(n_problems, g, lv, sh, nullptr);
    return batch_part(n_problems, lv, batch, part, sh, (hipStream_t)stream);
}

int imask_batch_step(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, void* batch,
                     int32_t n_steps, void* stream)
{
    if (int rc = batch_check(n_problems, g, lv)) return rc;
    if (!batch || n_steps < 0) return IMASK_EINVAL;
    StageShape sh;
    batch_shapes(n_problems, g, lv, sh, nullptr);
    for (int it = 0; it < n_steps; ++it)
        for (int part = IMASK_BATCH_PLAN; part <= IMASK_BATCH_ADVANCE; ++part)
            if (int rc = batch_part(n_problems, lv, batch, part, sh, (hipStream_t)stream)) return rc;
    return IMASK_OK;
}

static int batch_part(int n_problems, const imask_levels* lv, void* batch, int part, const StageShape& sh,
                      hipStream_t stream)
{
    const int n = n_problems;
    const BatchView bv = batch_view(batch, n, batch_rmax(n, lv));
    hipStream_t s = stream;
    auto stage = [&](int v, int j) -> int {
        if (sh.ub[v][j] <= 0) return IMASK_OK;
        const long long cap = 256LL * batch_wgs_per_cu(v, sh.lds[v][j]);
        const unsigned grid = (unsigned)std::max(1LL, std::min(sh.ub[v][j], cap));
        IMK_TRY(launch_batch_stage(v, j, bv, grid, sh.lds[v][j], s));
        return IMASK_OK;
    };
    // each phase runs its variants' slots in order: rounds, and within a
    // round the LDS classes
    auto phase = [&](int ph, int j0, int j1) -> int {
        for (int v = 0; v < kNumVariants; ++v)
            if (variant_phase(v) == ph)
                for (int j = j0; j < j1; ++j)
                    if (int rc = stage(v, j)) return rc;
        return IMASK_OK;
    };
    switch (part) {
    case IMASK_BATCH_PLAN:
        IMK_TRY(launch_batch_plan(bv, s));
        return IMASK_OK;
    case IMASK_BATCH_FORWARD:
        return phase(0, 0, kRounds);
    case IMASK_BATCH_TRANSPOSE:
        for (int r = 0; r < sh.rounds; ++r) {
            if (int rc = phase(1, r * kLdsClasses, (r + 1) * kLdsClasses)) return rc;
            if (int rc = phase(2, r * kLdsClasses, (r + 1) * kLdsClasses)) return rc;
        }
        return phase(3, 0, kRounds);
    default:
        IMK_TRY(launch_batch_advance(bv, s));
        return IMASK_OK;
    }
}

int imask_batch_state(int32_t n_problems, const imask_levels* lv, const void* batch, imask_state* s, void* stream)
{
    if (n_problems < 1 || n_problems > kMaxBatch || !lv || !batch || !s) return IMASK_EINVAL;
    std::vector<BatchProb> probs(n_problems);
    const BatchView bv = batch_view(const_cast<void*>(batch), n_problems, batch_rmax(n_problems, lv));
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(probs.data(), bv.prob, sizeof(BatchProb) * probs.size(), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return IMASK_EHIP;
    for (int q = 0; q < n_problems; ++q) {
        s[q].k = probs[q].k;
        s[q].cur = probs[q].cur;
        s[q].epochs = probs[q].epochs;
    }
    return IMASK_OK;
}

int imask_resample(int32_t n, int32_t log2f, int32_t mode, const imask_levels* lv, const float* in, float* out,
                   void* stream)
{
    imask_geometry g{n, 1, 1, 0.0, 0.0, 1.0, nullptr};
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

int imask_time_kernel(const imask_geometry* g, int32_t which, int32_t log2f, const void* work, const float* in,
                      float* out, int32_t reps, void* stream, double* avg_ms)
{
    if (!geometry_ok(g) || !work || !in || !out || !avg_ms || reps < 1) return IMASK_EINVAL;
    const Layout L = make_layout(*g);
    if (log2f < 0 || log2f > L.lmax) return IMASK_EINVAL;
    if (which != IMASK_KERNEL_FORWARD && which != IMASK_KERNEL_TRANSPOSE && which != IMASK_KERNEL_TRANSPOSE_SUM)
        return IMASK_EINVAL;
    float* W = (float*)work;
    hipStream_t s = (hipStream_t)stream;
    FwdArgs fa{};
    BpArgs ba{};
    if (which == IMASK_KERNEL_FORWARD) {
        // stage the restricted image once, then time the projector kernel alone
        if (int rc = imask_project(g, log2f, work, in, out, stream)) return rc;
        fwd_common(L, W, fa);
        fa.nterms = 1;
        fa.term[0] = FwdTerm{W + L.zp[log2f], W + L.zpT[log2f], log2f, 1.0f, W + L.fpart[log2f], L.fbands[log2f],
                             L.frows[log2f]};
    } else {
        ba.consts = (const RayConst*)(W + L.consts);
        ba.fan = fan_at(L, W);
        ba.split = split_at(L, W);
        ba.n = L.n;
        ba.na = L.na;
        ba.nd = L.nd;
        ba.lvl = log2f;
        ba.y = in;
        ba.out = out;
        ba.coef = 1.0f;
        ba.part = W + L.part;
        ba.tmp = W + L.ptmp;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return IMASK_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return IMASK_EHIP;
    }
    int rc = IMASK_OK;
    BpOwnArgs used;
    if (hipEventRecord(e0, s) != hipSuccess) rc = IMASK_EHIP;
    if (which == IMASK_KERNEL_TRANSPOSE_SUM) {
        ba.out = W + L.ptmp;  // the level image, not prolonged
        ba.tmp = W + L.ptmp;
    }
    for (int r = 0; r < reps && rc == IMASK_OK; ++r) {
        const hipError_t e = which == IMASK_KERNEL_FORWARD     ? launch_fwd_terms(fa, s)
                             : which == IMASK_KERNEL_TRANSPOSE ? launch_bp_main(ba, s, used)
                                                               : launch_bp(ba, s);
        if (e != hipSuccess) rc = IMASK_EHIP;
    }
    float ms = 0.0f;
    if (rc == IMASK_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = IMASK_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == IMASK_OK) *avg_ms = (double)ms / reps;
    return rc;
}

static int check_finite_after(int n_problems, const imask_geometry* g, const imask_params* prm,
                              const imask_state* s, hipStream_t st);

int imask_step_timed(const imask_geometry* g, const imask_levels* lv, const imask_reg* reg, const imask_params* prm,
                     const float* b, imask_state* s, int32_t n_steps, float* ms_out, void* stream)
{
    if (n_steps < 0 || (n_steps > 0 && !ms_out)) return IMASK_EINVAL;
    if (int rc = check_problem(g, lv, reg, prm, b, s)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const Layout L = make_layout(*g);
    std::vector<hipEvent_t> ev(n_steps + 1, nullptr);
    int rc = IMASK_OK;
    for (auto& e : ev)
        if (rc == IMASK_OK && hipEventCreate(&e) != hipSuccess) rc = IMASK_EHIP;
    if (rc == IMASK_OK && hipEventRecord(ev[0], st) != hipSuccess) rc = IMASK_EHIP;
    PrepCarry carry;
    for (int it = 0; it < n_steps && rc == IMASK_OK; ++it) {
        rc = one_step(*g, L, *lv, *reg, *prm, b, *s, st, &carry, it + 1 < n_steps);
        if (rc == IMASK_OK && hipEventRecord(ev[it + 1], st) != hipSuccess) rc = IMASK_EHIP;
    }
    if (rc == IMASK_OK && n_steps > 0 && hipEventSynchronize(ev[n_steps]) != hipSuccess) rc = IMASK_EHIP;
    for (int it = 0; it < n_steps && rc == IMASK_OK; ++it)
        if (hipEventElapsedTime(&ms_out[it], ev[it], ev[it + 1]) != hipSuccess) rc = IMASK_EHIP;
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc != IMASK_OK) return rc;
    return check_finite_after(1, g, prm, s, st);
}

size_t imask_constants_scratch_bytes(const imask_geometry* g)
{
    if (!geometry_ok(g)) return 0;
    const size_t d = (size_t)g->n * g->n, m = (size_t)g->n_angles * g->n_det;
    return (3 * d + 3 * m) * sizeof(float) + (kConstDotDoubles) * sizeof(double);
}

}  // extern "C"

namespace {

// Buffers of the power method, carved from the caller's scratch.
struct PowerBufs {
    float *x, *xs, *xt;  // image vectors
    float *y, *ys, *yt;  // sinogram vectors
    double* part;        // dot partials
    double* dot;         // one dot result
};

struct PowerCtx {
    const imask_geometry* g;
    const imask_levels* lv;
    const void* work;
    hipStream_t s;
    PowerBufs b;
    size_t d, m;
};

int sk(PowerCtx& c, int k, int adj, const float* in, float* out)
{
    return imask_sketch_apply(c.g, c.lv, k, adj, c.work, in, out, (void*)c.s);
}

int zero(float* p, size_t n, hipStream_t s) { return launch_fill(p, n, 0.0f, s) == hipSuccess ? IMASK_OK : IMASK_EHIP; }

// out = sum_k w_k K_k^T K_k v (image side) or sum_k w_k K_k K_k^T v (sinogram side)
int gram(PowerCtx& c, bool image_side, const double* w, const float* v, float* out)
{
    const size_t no = image_side ? c.d : c.m;
    if (int rc = zero(out, no, c.s)) return rc;
    float* mid = image_side ? c.b.ys : c.b.xs;
    float* t = image_side ? c.b.xt : c.b.yt;
    for (int k = 0; k < c.lv->r; ++k) {
        if (int rc = sk(c, k, image_side ? 0 : 1, v, mid)) return rc;
        if (int rc = sk(c, k, image_side ? 1 : 0, mid, t)) return rc;
        if (launch_axpy(out, t, (float)w[k], no, c.s) != hipSuccess) return IMASK_EHIP;
    }
    return IMASK_OK;
}

// out = Kbar^T Kbar v, Kbar = sum_k p_k K_k
int kbar_gram(PowerCtx& c, const float* v, float* out)
{
    if (int rc = zero(c.b.ys, c.m, c.s)) return rc;
    for (int k = 0; k < c.lv->r; ++k) {
        if (int rc = sk(c, k, 0, v, c.b.yt)) return rc;
        if (launch_axpy(c.b.ys, c.b.yt, (float)c.lv->p[k], c.m, c.s) != hipSuccess) return IMASK_EHIP;
    }
    if (int rc = zero(out, c.d, c.s)) return rc;
    for (int k = 0; k < c.lv->r; ++k) {
        if (int rc = sk(c, k, 1, c.b.ys, c.b.xt)) return rc;
        if (launch_axpy(out, c.b.xt, (float)c.lv->p[k], c.d, c.s) != hipSuccess) return IMASK_EHIP;
    }
    return IMASK_OK;
}

int dot_host(PowerCtx& c, const float* a, const float* b, size_t n, double* out)
{
    if (launch_dot(a, b, n, c.b.part, c.b.dot, c.s) != hipSuccess) return IMASK_EHIP;
    if (hipMemcpyAsync(out, c.b.dot, sizeof(double), hipMemcpyDeviceToHost, c.s) != hipSuccess) return IMASK_EHIP;
    if (hipStreamSynchronize(c.s) != hipSuccess) return IMASK_EHIP;
    return IMASK_OK;
}

// Largest eigenvalue of a symmetric PSD operator by the power method:
// lambda = <v, A v> with v normalised, `iters` times.
template <class Op>
int power(PowerCtx& c, float* v, float* w, size_t n, int iters, unsigned long long seed, Op op, double* lam)
{
    if (launch_fill_random(v, n, seed, c.s) != hipSuccess) return IMASK_EHIP;
    double nrm2 = 0.0;
    if (int rc = dot_host(c, v, v, n, &nrm2)) return rc;
    if (launch_scale(v, (float)(1.0 / std::sqrt(nrm2)), n, c.s) != hipSuccess) return IMASK_EHIP;
    *lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        if (int rc = op(v, w)) return rc;
        if (int rc = dot_host(c, v, w, n, lam)) return rc;
        if (int rc = dot_host(c, w, w, n, &nrm2)) return rc;
        if (!(nrm2 > 0.0)) {
            *lam = 0.0;
            return IMASK_OK;
        }
        std::swap(v, w);
        if (launch_scale(v, (float)(1.0 / std::sqrt(nrm2)), n, c.s) != hipSuccess) return IMASK_EHIP;
    }
    return IMASK_OK;
}

}  // namespace

extern "C" {

int imask_step_constants(const imask_geometry* g, const imask_levels* lv, double mu, int32_t iters, uint64_t seed,
                         const void* work, void* scratch, double* out_host, void* stream)
{
    if (!geometry_ok(g) || !work || !scratch || !out_host || iters < 1 || !(mu > 0.0)) return IMASK_EINVAL;
    if (!levels_ok(lv, level_limit(g->n))) return IMASK_EINVAL;
    PowerCtx c;
    c.g = g;
    c.lv = lv;
    c.work = work;
    c.s = (hipStream_t)stream;
    c.d = (size_t)g->n * g->n;
    c.m = (size_t)g->n_angles * g->n_det;
    double* dd = (double*)scratch;
    c.b.part = dd;
    c.b.dot = dd + kDotPartials;
    float* f = (float*)(dd + kConstDotDoubles);
    c.b.x = f;
    c.b.xs = f + c.d;
    c.b.xt = f + 2 * c.d;
    c.b.y = f + 3 * c.d;
    c.b.ys = c.b.y + c.m;
    c.b.yt = c.b.ys + c.m;
    double p[IMASK_MAX_LEVELS], p2[IMASK_MAX_LEVELS];
    for (int k = 0; k < lv->r; ++k) {
        p[k] = lv->p[k];
        p2[k] = lv->p[k] * lv->p[k];
    }
    // iterates alternate x <-> xs (image side) and y <-> ys (sinogram side);
    // the operators' temporaries are ys, yt, xt (image side) and xs, yt
    // (sinogram side), disjoint from the iterates they work on
    float* xv = c.b.x;
    float* yv = c.b.y;
    double l2 = 0, lbx = 0, lby = 0, lpx = 0, lpy = 0;
    {
        auto op = [&](const float* v, float* w) { return kbar_gram(c, v, w); };
        if (int rc = power(c, xv, c.b.xs, c.d, iters, seed ^ 0x1ULL, op, &l2)) return rc;
    }
    {
        auto op = [&](const float* v, float* w) { return gram(c, true, p2, v, w); };
        if (int rc = power(c, xv, c.b.xs, c.d, iters, seed ^ 0x2ULL, op, &lbx)) return rc;
    }
    {
        auto op = [&](const float* v, float* w) { return gram(c, true, p, v, w); };
        if (int rc = power(c, xv, c.b.xs, c.d, iters, seed ^ 0x3ULL, op, &lpx)) return rc;
    }
    {
        auto op = [&](const float* v, float* w) { return gram(c, false, p2, v, w); };
        if (int rc = power(c, yv, c.b.ys, c.m, iters, seed ^ 0x4ULL, op, &lby)) return rc;
    }
    {
        auto op = [&](const float* v, float* w) { return gram(c, false, p, v, w); };
        if (int rc = power(c, yv, c.b.ys, c.m, iters, seed ^ 0x5ULL, op, &lpy)) return rc;
    }
    out_host[0] = l2 / mu;
    out_host[1] = std::max(lbx, lby) / mu;
    out_host[2] = std::max(lpx, lpy) / mu;
    return IMASK_OK;
}

int imask_sigma_balamurugan(double L2, double Lbar2, double* sigma_out)
{
    if (!(L2 > 0) || !(Lbar2 > 0) || !std::isfinite(L2) || !std::isfinite(Lbar2) || !sigma_out) return IMASK_EINVAL;
    *sigma_out = 1.0 / (L2 + 3.0 * Lbar2);
    return IMASK_OK;
}

int imask_sigma_thm3(double L2, double Lbar2, double Lbarp2, double pmin, int32_t grid, double* sigma_out,
                     double* theta_out)
{
    if (!(L2 > 0) || !(Lbar2 > 0) || !(Lbarp2 > 0) || !(pmin > 0 && pmin <= 1) || grid < 2 || !sigma_out)
        return IMASK_EINVAL;
    const double cbar = 1.0 / (1.0 + L2 + Lbarp2);
    double best_theta = 2.0, best_eta = 0.0;
    for (int ic = 1; ic <= grid; ++ic) {
        const double c = cbar * ic / (grid + 1.0);
        for (int ir = 1; ir <= grid; ++ir) {
            const double rho = ir / (grid + 1.0);
            // alpha^{-1} (eq. (alpha)); phi and psi of Sec. 3.5
            const double ainv = (Lbar2 / (rho * c)) * (1.0 - (1.0 + L2) * c) / (1.0 - (1.0 + L2 + Lbarp2) * c);
            double eta, theta;
            if (pmin > ainv * c * c + (1.0 - rho) * c) {  // eq. (opt:cond): eta* = c
                eta = c;
                theta = 1.0 - (1.0 - rho) * c;
            } else {  // eq. (eta_opt): phi(eta) = psi(eta)
                const double q = ainv - 1.0 / c;
                eta = std::fabs(q) < 1e-300 ? 0.5 * (pmin + rho * c)
                                            : (std::sqrt(1.0 + q * (pmin + rho * c)) - 1.0) / q;
                theta = (eta - c) * (eta - c) / c + 1.0 - (1.0 - rho) * c;
            }
            if (theta < best_theta) {
                best_theta = theta;
                best_eta = eta;
            }
        }
    }
    *sigma_out = best_eta / (1.0 - best_eta);
    if (theta_out) *theta_out = best_theta;
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
    if (!(prm->sigma > 0.0) || !std::isfinite(prm->sigma) || prm->reserved != 0) return IMASK_EINVAL;
    if (reg->kind == IMASK_REG_TV && (!s->tvd[0] || !s->tvd[1] || s->tvd[0] == s->tvd[1])) return IMASK_EINVAL;
    if (s->ztab) {
        if (s->ztab == s->phi || s->ztab == s->psi || s->ztab == s->x[0] || s->ztab == s->x[1]) return IMASK_EINVAL;
        if (prm->schedule != IMASK_SCHEDULE_PARALLEL) return IMASK_ENOTSUP;
    }
    if (prm->draw_mode == IMASK_DRAW_INDEPENDENT) {
        if (prm->schedule != IMASK_SCHEDULE_PARALLEL || s->ztab) return IMASK_ENOTSUP;
    } else if (prm->draw_mode != IMASK_DRAW_COMMON) {
        return IMASK_EINVAL;
    }
    if (lv->n_blocks > g->n_angles) return IMASK_EINVAL;
    if (lv->n_blocks > 1 && (prm->schedule != IMASK_SCHEDULE_PARALLEL || s->ztab ||
                             prm->draw_mode != IMASK_DRAW_COMMON || g->angles))
        return IMASK_ENOTSUP;
    if (prm->schedule == IMASK_SCHEDULE_SEQUENTIAL) {
        if (!(prm->theta >= 0.0 && prm->theta <= 1.0) || !s->xbar) return IMASK_EINVAL;
        if (s->xbar == s->x[0] || s->xbar == s->x[1]) return IMASK_EINVAL;
    } else if (prm->schedule != IMASK_SCHEDULE_PARALLEL) {
        return IMASK_EINVAL;
    }
    return IMASK_OK;
}

// The opt-in finiteness test of x and y after a call's last step (one
// synchronisation for all problems that ask for it).
static int check_finite_after(int n_problems, const imask_geometry* g, const imask_params* prm,
                              const imask_state* s, hipStream_t st)
{
    std::vector<int> flags(n_problems, 0);
    bool any = false;
    for (int q = 0; q < n_problems; ++q) {
        if (!prm[q].check_finite) continue;
        const Layout L = make_layout(g[q]);
        int* flag = (int*)((float*)s[q].work + L.flag);
        IMK_TRY(launch_nonfinite(s[q].x[s[q].cur], (size_t)g[q].n * g[q].n, s[q].y[s[q].cur],
                                 (size_t)g[q].n_angles * g[q].n_det, flag, st));
        if (hipMemcpyAsync(&flags[q], flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return IMASK_EHIP;
        any = true;
    }
    if (!any) return IMASK_OK;
    if (hipStreamSynchronize(st) != hipSuccess) return IMASK_EHIP;
    for (int q = 0; q < n_problems; ++q)
        if (flags[q]) return IMASK_ENONFINITE;
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
    std::vector<PrepCarry> carry(n_problems);
    for (int it = 0; it < n_steps; ++it)
        for (int q = 0; q < n_problems; ++q) {
            const Layout L = make_layout(g[q]);
            if (int rc = one_step(g[q], L, lv[q], reg[q], prm[q], b[q], s[q], st, &carry[q], it + 1 < n_steps))
                return rc;
        }
    return check_finite_after(n_problems, g, prm, s, st);
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
        PrepCarry carry;
        for (;;) {
            const bool done = budget_kind == IMASK_BUDGET_ITERS ? (double)(s[q].k - k_start) >= budget
                                                                : s[q].epochs - e_start >= budget;
            if (done) break;
            // with an epoch budget the step after this one may not run; a
            // restriction carried for it is then left unused
            const bool more = budget_kind == IMASK_BUDGET_EPOCHS || (double)(s[q].k + 1 - k_start) < budget;
            if (int rc = one_step(g[q], L, lv[q], reg[q], prm[q], b[q], s[q], st, &carry, more)) return rc;
        }
    }
    return check_finite_after(n_problems, g, prm, s, st);
}

}  // extern "C"
