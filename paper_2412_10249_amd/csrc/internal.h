// internal.h - launch interface between the C ABI (api.hip) and the gfx950
// kernels (kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

#include "imask.h"

namespace imk {

// Projector constants of one (level, angle).  The interpolation coordinate
// of ray b at step i (row for row-stepping angles, column otherwise) is the
// exact fixed-point value u = cfx + i*afx + b*bfx in units of 2^-32 pixel:
// its high word is the left tap j0 and its low word the weight of the right
// tap.  Both projector directions use this integer formula, so they agree on
// every weight bit for bit.  The float fields mirror it for range estimates;
// w is the step length h_l/|cos| (or h_l/|sin|), ib = 1/b.
struct RayConst {
    long long afx, bfx, cfx;
    int phases;  // ceil(2^32/|bfx|): rays this far apart never share a tap
    int pad;
    float a, b, c, w, ib, r0, r1, r2;
};
static_assert(sizeof(RayConst) == 64, "RayConst is 64 bytes");
constexpr int kConstStride = 16;  // floats per RayConst
// Zero columns around every padded image row: kPadL before, kPadL after.
#ifndef IMK_PART_IMAGES
#define IMK_PART_IMAGES 16
#endif
// Full-resolution partial images the transpose may write (2 G N_l^2 <= this * N^2).
constexpr int kPartImages = IMK_PART_IMAGES;
// Partial images of the parallel-beam transposes: up to kParPartImages N^2
// floats while that stays within kParPartFloats, so that small grids get
// more angle groups (512^2: 32 partial images, about 2048 workgroups at
// level 0), never fewer than kPartImages N^2.
constexpr int kParPartImages = 64;
constexpr size_t kParPartFloats = (size_t)8 << 20;  // 32 MiB
// Partial images of the fan transposes: up to kFanPartImages N^2 floats
// while that stays within kFanPartFloats (more view groups where rays are
// few per workgroup), never fewer than kPartImages N^2.
constexpr int kFanPartImages = 64;
constexpr size_t kFanPartFloats = (size_t)64 << 20;  // 256 MiB
constexpr int kPadL = 4;
constexpr int kPad = 2 * kPadL;

// Angle lists of the two stepping directions.  Default angles a*pi/na:
// the row-stepping angles are s0a..s0a+n0a-1 and s0b..s0b+(nrow-n0a)-1, the
// column-stepping ones s1..s1+ncol-1 (for all angles: 0..n_lo-1 and
// a_hi0..na-1, and n_lo..a_hi0-1; a measurement block takes the part of
// each range inside its angles).  Listed angles: perm (device) holds the
// nrow row-stepping angle indices, then the ncol column-stepping ones, each
// ascending, and rows[a] (device) is 1 for a row-stepping angle; both are
// null by default.
struct AngleSplit {
    int s0a, n0a, s0b, nrow, s1, ncol;
    const int* perm;
    const int* rows;
};
inline AngleSplit angle_split(int na)
{
    int n_lo = na / 4 + 1;
    int a_hi0 = (3 * na + 3) / 4;
    if (n_lo > na) n_lo = na;
    if (a_hi0 < n_lo) a_hi0 = n_lo;
    AngleSplit s{};
    s.s0a = 0;
    s.n0a = n_lo;
    s.s0b = a_hi0;
    s.nrow = n_lo + (na - a_hi0);
    s.s1 = n_lo;
    s.ncol = a_hi0 - n_lo;
    return s;
}
// The default angles a0..a1-1 (a measurement block) split the same way.
inline AngleSplit angle_split_range(int na, int a0, int a1)
{
    const AngleSplit f = angle_split(na);
    auto clip = [](int lo, int hi, int b0, int b1, int* start) {
        *start = lo > b0 ? lo : b0;
        const int end = hi < b1 ? hi : b1;
        return end > *start ? end - *start : 0;
    };
    AngleSplit s{};
    int nb;
    s.n0a = clip(f.s0a, f.s0a + f.n0a, a0, a1, &s.s0a);
    nb = clip(f.s0b, na, a0, a1, &s.s0b);
    s.nrow = s.n0a + nb;
    s.ncol = clip(f.s1, f.s1 + f.ncol, a0, a1, &s.s1);
    return s;
}

// Fan-beam ray (one per view and bin), its line x ct + y st = s in the form
// the Joseph walk needs.  For a row-stepping ray (|ct| >= |st|) the column
// coordinate at row i of level l (pixel size h) is
//   u(i) = (P + (E - h/2)(T + 1)) / h - i T,   P = s/ct, T = st/ct,
// and the step length is h sec, sec = 1/|ct|; a column-stepping ray is the
// mirror (P = s/st, T = ct/st, sec = 1/|st|, rows and columns swapped).
// Both kernels of the pair turn these doubles into the same fixed-point
// coordinate with fan_coords, so they agree on every weight bit for bit.
struct FanRay {
    double P, T, sec;
    int row;
    int pad;
};
static_assert(sizeof(FanRay) == 32, "FanRay is 32 bytes");
// Fan-beam view: cos and sin of the source angle beta, and whether any of
// its rays step along rows / along columns.
struct FanView {
    double c, s;
    int has_row, has_col;
    int pad[2];
};
static_assert(sizeof(FanView) == 32, "FanView is 32 bytes");
// A fan ray on one level, as the transpose scatters it: the fixed-point
// coordinate u(step) = cfx + step * afx (from fan_coords), the weighted datum
// w_ray * y, and the stepping axis.
struct FanTab {
    long long cfx, afx;
    float wy;
    int row;
};
static_assert(sizeof(FanTab) == 24, "FanTab is 24 bytes");
// What the fan kernels need besides the ray and view tables: the domain
// half side, source and detector distances, bin spacing and offset.
struct FanGeo {
    const FanRay* ray;    // n_angles x n_det, view-major; null: parallel beam
    const FanView* view;  // n_angles
    FanTab* tab;          // n_angles x n_det, the transpose's per-launch table
    double E, D, Dd, ds, s0;
    double min_sep;       // lower bound of adjacent rays' separation (domain units)
    float bmargin;        // bins added to each side of an FP32 bin estimate
    int va, vb;           // the views a launch covers (a measurement block), else all
    long long part_floats;  // size of the partial-image buffer (floats)
};

// Workspace layout for one geometry (offsets in floats from the start).
struct Layout {
    int n = 0, na = 0, nd = 0, lmax = 0;
    size_t consts = 0;
    size_t zp[IMASK_MAX_LOG2F + 1] = {};   // padded level-l image, rows
    size_t zpT[IMASK_MAX_LOG2F + 1] = {};  // padded level-l image, transposed
    size_t craw[IMASK_MAX_LOG2F + 1] = {}; // raw level-l backprojection N_l^2
    size_t vbuf = 0;                       // N^2 prox input
    size_t part = 0;                       // kPartImages N^2 per-angle-group partial backprojections
    size_t ptmp = 0;                       // N^2 coarse result before prolongation
    size_t fpart[IMASK_MAX_LOG2F + 1] = {};// per-band partial projections, fwd_bands(l) * m
    int fbands[IMASK_MAX_LOG2F + 1] = {};  // row bands of the level-l forward
    int frows[IMASK_MAX_LOG2F + 1] = {};   // rows per band (0: direct kernel, one band)
    // listed angles: na doubles (radians), then perm and rows (na int32 each)
    size_t angtab = 0;
    size_t flag = 0;                       // int flag of the finiteness check
    int listed = 0;
    AngleSplit split{};                    // perm / rows unset: see split_at
    // fan beam: ray table (m FanRay) and view table (na FanView)
    int fan = 0;
    size_t fray = 0, fview = 0, ftab = 0;
    size_t part_floats = 0;  // size of the partial-image buffer
    double E = 1.0, D = 0.0, Dd = 0.0, ds = 0.0, s0 = 0.0, bmargin = 0.0, min_sep = 0.0;
    size_t total = 0;
};

Layout make_layout(const imask_geometry& g);
// The layout's angle split with its device tables in workspace W.
inline AngleSplit split_at(const Layout& L, const float* W)
{
    AngleSplit s = L.split;
    if (L.listed) {
        const int* t = (const int*)(W + L.angtab + 2 * (size_t)L.na);
        s.perm = t;
        s.rows = t + L.na;
    }
    return s;
}
inline FanGeo fan_at(const Layout& L, const float* W)
{
    FanGeo f{};
    if (L.fan) {
        f.ray = (const FanRay*)(W + L.fray);
        f.view = (const FanView*)(W + L.fview);
        f.tab = (FanTab*)(const_cast<float*>(W) + L.ftab);
    }
    f.E = L.E;
    f.D = L.D;
    f.Dd = L.Dd;
    f.ds = L.ds;
    f.s0 = L.s0;
    f.bmargin = (float)L.bmargin;
    f.min_sep = L.min_sep;
    f.va = 0;
    f.vb = L.na;
    f.part_floats = (long long)L.part_floats;
    return f;
}
inline int side(int n, int l) { return n >> l; }
inline int pstride(int n, int l) { return (n >> l) + kPad; }

// ---- kernels' argument blocks (passed by value) ----

enum { FWD_STORE = 0, FWD_ACCUM = 1, FWD_DUAL = 2 };

struct FwdTerm {
    const float* img;   // padded rows of the level image
    const float* imgT;  // padded transposed level image
    int lvl;
    float coef;
    float* part;        // this level's per-band partial projections
    int bands, rows;    // band layout (rows == 0: one band, direct kernel)
};

struct FwdArgs {
    const RayConst* consts;
    FanGeo fan;
    AngleSplit split;
    int n, na, nd;
    int nterms;
    FwdTerm term[IMASK_MAX_LEVELS];
    int mode;
    float* out;
    // dual SAGA epilogue
    const float* y_old;
    const float* bdat;
    float* y_new;
    float* psi;   // r tables, or the running average when compact
    int r, kidx, compact;
    float p[IMASK_MAX_LEVELS];
    float sigma, inv1ps;
    // sinogram elements [e0, e1) hold this step's measurement block: outside
    // it the projection is zero and psi is not refreshed (all of m by default)
    long long e0, e1;
};

struct FwdBandArgs {
    const RayConst* consts;
    FanGeo fan;
    int n, na, nd, lvl;
    const float* img;
    const float* imgT;
    float* part;
    int R, bands, apg, groups_row, groups_col;
    AngleSplit split;
    // single band and single term: the dual step of Alg. 1 in the epilogue
    // (the reduce's arithmetic, element by element; no partial is written)
    int dual;
    const float* y_old;
    const float* bdat;
    float* y_new;
    float* psi;
    int r, kidx;
    float p[IMASK_MAX_LEVELS];
    float sigma, inv1ps;
};

struct BpOwnArgs {
    const RayConst* consts;
    FanGeo fan;
    int n, na, nd, lvl;
    int wave_range;  // each wavefront takes the bins of its own rows (else the workgroup's)
    int tab;         // angles a workgroup tabulates in LDS at once (0: the largest table)
    const float* y;
    float* part;  // nq partial images N_l x N_l, image orientation
    int G;
    int nq;     // partial images to sum (2 G: both passes)
    AngleSplit split;
    float* out;
    float coef;
    int accumulate, prolong;
};

struct BpArgs {
    const RayConst* consts;
    FanGeo fan;
    AngleSplit split;
    int n, na, nd, lvl;
    const float* y;
    float* out;
    float coef;
    int accumulate;
    int prolong;  // 1: write the 2^l x 2^l block of an N x N image
    float* part;  // per-angle-group partial sums (16 N^2 floats of workspace)
    float* tmp;   // N_l^2 scratch for the prolonged store
};

enum { PREP_MEAN = 0, PREP_COMP = 1 };

struct PrepOut {
    float* dst;
    float* dstT;  // may be null
    int lvl;
    int kind;
    int padded;
};

struct PrepArgs {
    const float* x;
    // compact dual tables: the restricted input is taken relative to this
    // snapshot (level snap_lvl, N_l^2), which is then replaced by it
    float* snap;
    int snap_lvl;
    int n, T, pyr_levels;
    int nout;
    PrepOut out[IMASK_MAX_LEVELS + 1];
    int ncomp;
    int comp_lvl[IMASK_MAX_LEVELS];
    float comp_p[IMASK_MAX_LEVELS];
    float inv_p0;
};

struct PrimalArgs {
    int n, T, pyr_levels;
    int r, kidx, full_mode;
    int lvl[IMASK_MAX_LEVELS];
    float p[IMASK_MAX_LEVELS];
    const float* craw[IMASK_MAX_LEVELS];
    float* phi;
    long long phi_off[IMASK_MAX_LEVELS];
    const float* x_old;
    float* x_out;
    float tau, prox_scale;
    float* xbar;  // when set: xbar = x_out + theta (x_out - x_old)
    float theta;
    // measurement blocks: phi holds nblk copies of the r tables, block b's
    // at b * blk_stride; this step refreshes block jblk's table kidx.  The
    // table average weighs table (c, b) by pavg[c] = p[c] / nblk; p itself
    // builds the sketches (compensation, UNBIASED combination)
    int nblk, jblk;
    long long blk_stride;
    float pavg[IMASK_MAX_LEVELS];
};

struct TvArgs {
    int n, J;
    const float* v;
    const float* u0;
    float* out;
    float* xbar;  // when set: xbar = out + theta (out - u0)
    float theta;
    float tau_w, tau_lam, eps, invL;
    float beta[IMASK_MAX_TV_INNER];
    // when set: the restriction k_prep would make of `out` for the next
    // step, written by the prox's epilogue (only where tv_prep_fusable)
    int prep_next;
    PrepArgs next;
};
// Whether the smoothed-TV prox can write these restricted copies of its
// output itself: whole tiles, every level inside a tile, no snapshot.
bool tv_prep_fusable(int n, const PrepArgs& pa);

// Forward band layout of a level with nl pixels per side (LDS-resident
// bands of rows); rows == 0 selects the direct (global-memory) kernel.
// fwd_bands_default is the layout the workspace is sized for; fwd_bands
// the one the launches use (the tuned LDS budget, never more bands).
void fwd_bands_default(int nl, int na, int nd, int* bands, int* rows);
void fwd_bands(int nl, int na, int nd, int* bands, int* rows);

// Tunable launch shapes of the levels of one grid side and detector
// (imask_set_tiles); zero fields select the defaults.
struct Tiles {
    int bp_rows = 0, bp_waves = 0;  // transpose tile: rows per wavefront, wavefronts
    int bp_wg = 0;                  // transpose workgroup target
    int fwd_lds_kb = 0;             // forward band LDS budget (KB)
};
Tiles tiles_for(int nl, int na, int nd);
bool set_tiles(int nl, int na, int nd, const Tiles* t);  // null resets; false: unsupported shape

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_consts(const imask_geometry& g, const Layout& L, float* work, hipStream_t s);
hipError_t launch_fill(float* p, size_t count, float value, hipStream_t s);
// *flag = 1 if a[0..na) or b[0..nb) holds a NaN or an infinity, else 0
hipError_t launch_nonfinite(const float* a, size_t na, const float* b, size_t nb, int* flag, hipStream_t s);
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
hipError_t launch_fwd(const FwdArgs& a, hipStream_t s);        // projector kernels + reduce/epilogue
hipError_t launch_fwd_terms(const FwdArgs& a, hipStream_t s);  // projector kernels only
hipError_t launch_bp(const BpArgs& a, hipStream_t s);          // transpose kernel + ordered sum
hipError_t launch_bp_main(const BpArgs& a, hipStream_t s, BpOwnArgs& used);  // transpose kernel only
hipError_t launch_primal(const PrimalArgs& a, hipStream_t s);
// Transpose at level ba.lvl, its ordered partial sum and the primal step in
// one epilogue kernel (steps whose sketch needs a single backprojection).
hipError_t launch_bp_primal(const BpArgs& ba, const PrimalArgs& pr, hipStream_t s);
hipError_t launch_tv(const TvArgs& a, hipStream_t s);

// Prox of gamma TV + nonnegativity at v / scale by J dual FGP iterations.
struct TvdArgs {
    int n, J;
    const float* v;       // prox input (before the 1/scale)
    const float* pin;     // dual pair in (2 n^2)
    float* pout;          // dual pair out (2 n^2)
    float* out;           // x^{k+1}
    const float* u0;      // x^k, for the extrapolation
    float* xbar;          // when set: xbar = out + theta (out - u0)
    float theta;
    float inv_scale, gamma, inv8g;
    float beta[IMASK_MAX_TV_INNER];
};
hipError_t launch_tvd(const TvdArgs& a, hipStream_t s);
hipError_t launch_prolong(const float* in, float* out, int n, int lvl, float coef, hipStream_t s);
hipError_t launch_project_block(const float* in, float* out, int n, int lvl, hipStream_t s);

hipError_t launch_axpy(float* y, const float* x, float a, size_t n, hipStream_t s);
hipError_t launch_scale(float* x, float a, size_t n, hipStream_t s);
hipError_t launch_fill_random(float* x, size_t n, unsigned long long seed, hipStream_t s);
// out = sum a[q] b[q] in FP64 (256 block partials in `part`, then one block)
hipError_t launch_dot(const float* a, const float* b, size_t n, double* part, double* out, hipStream_t s);

// pyramid tile side used by prep/primal for a set of levels up to lmax
int tile_side(int n, int lmax);

// ---- the launches of a step as data ----
//
// The parallel-beam launchers describe each kernel launch as a record
// (kernel variant, grid, block, dynamic LDS and the argument block) and then
// launch the records; the batched path stores the same records for many
// problems on the device and runs each variant once for all of them, so a
// problem gets the same launches, shapes and arguments either way.
enum Variant {
    V_PREP = 0,
    V_FWD_BAND,
    V_FWD_DIRECT,
    V_RED4,
    V_RED1,
    V_BP28,  // k_bp_own<2, 8>
    V_BP44,  // k_bp_own<4, 4>
    V_BP14,  // k_bp_own<1, 4>
    V_BP12,  // k_bp_own<1, 2>
    V_BP24,  // k_bp_own<2, 4>
    V_SUM4,
    V_SUM1,
    V_SUMP4,
    V_SUMP1,
    V_PRIMAL,
    V_SUMPT,  // level 0's ordered partial sum with the tile primal step (PAPER sketches)
    kNumVariants,
    // single-problem launches over several levels at once (the UNBIASED
    // full-resolution sketch); the batched path runs levels together anyway
    V_FWD_MULTI = kNumVariants,
    V_BP_MULTI28,
    V_BP_MULTI44,
    V_SUM_MULTI,
    // a transpose with the forward's band reduce in its last workgroups
    // (the two are independent in Alg. 1's parallel schedule)
    V_BPRED28,
    V_BPRED44,
    V_BPRED14,
    V_BPRED12,
    V_BPRED24,
    // a transpose with a single-band forward (dual step in its epilogue) in
    // its last workgroups (independent in the parallel schedule)
    V_BPFWD28,
    V_BPFWD44,
    V_BPFWD14,
    V_BPFWD12,
    V_BPFWD24
};
constexpr int kLaunchArgBytes = 3072;
constexpr int kBlobBytes = 640;  // argument blocks of the batched variants

// Several levels in one launch: block b belongs to part t when
// start[t] <= b < start[t + 1], and is block b - start[t] of that part's own
// grid (gx[t] blocks in x).
struct FwdMultiArgs {
    int n;
    int start[IMASK_MAX_LEVELS + 1];
    int gx[IMASK_MAX_LEVELS];
    FwdBandArgs t[IMASK_MAX_LEVELS];
};
struct BpMultiArgs {
    int n;
    int start[IMASK_MAX_LEVELS + 1];
    int gx[IMASK_MAX_LEVELS];
    BpOwnArgs t[IMASK_MAX_LEVELS];
};

// k_bp_sum / k_bp_sum_primal argument blocks.
struct SumArgs {
    BpOwnArgs a;
    float* tmp;
    int S;
};
struct SumPrimalArgs {
    BpOwnArgs a;
    PrimalArgs p;
    int S;
};
struct SumTileArgs {
    BpOwnArgs a;
    PrimalArgs p;
};
// Blocks [0, nbp) of the launch are the transpose's (its grid bgx x (nbp /
// bgx)), blocks [nbp, nbp + nred) the reduce's (16-byte accesses if red4).
struct BpRedArgs {
    BpOwnArgs b;
    FwdArgs f;
    int nbp, bgx, nred, red4;
};
// Blocks [0, nfwd) a single-band forward's (grid fgx x (nfwd / fgx)), the
// rest the transpose's (grid bgx x (nbp / bgx)).
struct BpFwdArgs {
    BpOwnArgs b;
    FwdBandArgs f;
    int nbp, bgx, nfwd, fgx;
};
struct SumMultiArgs {
    int n;
    int start[IMASK_MAX_LEVELS + 1];
    int v[IMASK_MAX_LEVELS];  // cells per thread of each part (4 or 1)
    SumArgs t[IMASK_MAX_LEVELS];
};

struct Launch {
    int variant = 0;
    int round = 0;  // transposes of a step share the partial images: round j runs after round j-1's sum
    unsigned gx = 1, gy = 1, gz = 1;
    int block = 0, lds = 0;
    alignas(16) unsigned char args[kLaunchArgBytes];
    template <class T>
    void set(const T& t)
    {
        static_assert(sizeof(T) <= kLaunchArgBytes, "argument block too large");
        std::memcpy(args, &t, sizeof(T));
    }
    template <class T>
    const T& get() const
    {
        return *reinterpret_cast<const T*>(args);
    }
};
using Launches = std::vector<Launch>;

// Records of the parallel-beam launchers (fan-beam geometries are not
// described this way).
void plan_prep(const PrepArgs& a, Launches& out);
void plan_fwd_terms(const FwdArgs& a, Launches& out);
void plan_fwd(const FwdArgs& a, Launches& out);                 // terms + reduce / dual step
void plan_bp_main(const BpArgs& ba, int round, Launches& out, BpOwnArgs* used);
void plan_bp(const BpArgs& ba, int round, Launches& out);       // transpose + ordered sum (no prolongation)
void plan_bp_primal(const BpArgs& ba, const PrimalArgs& pr, Launches& out);
void plan_primal(const PrimalArgs& a, Launches& out);
// Level 0's ordered sum of the partial images `a` wrote, fused with the
// primal step of a PAPER full-resolution sketch (one workgroup per 32 x 32
// tile), where sum_primal_tile_fits: N a multiple of 32, levels down to 32.
bool sum_primal_tile_fits(const PrimalArgs& pr);
void plan_sum_primal_tile(const BpOwnArgs& a, const PrimalArgs& pr, Launches& out);
// Moves the step's band reduce (a V_RED4 / V_RED1 record) into the first
// transpose launch after it, as extra workgroups; single-problem steps of
// the parallel schedule only (the transpose reads the old dual iterate).
void merge_reduce_into_transpose(Launches& out);
// Moves a single-band forward with the dual step in its epilogue into the
// first transpose launch after it (same conditions).
void merge_forward_into_transpose(Launches& out);
// The terms of an UNBIASED full-resolution sketch: every band-layout forward
// term in one launch (direct terms launched alone), and the coarse levels'
// transposes in one launch per tile shape with their partial images side by
// side in the workspace buffer, then their ordered sums in one launch.
void plan_fwd_fused(const FwdArgs& a, Launches& out);
// The coarse transposes with their partial images side by side in the
// buffer (groups reduced to fit); `fused`: one launch per tile shape and
// one for the sums, else (or when a level's tile has no fused form) the
// same transposes and sums as separate records of `round`.  Returns
// whether the fused launches were used.
bool plan_bp_coarse(const BpArgs* ba, int n, size_t part_floats, bool fused, int round, Launches& out);
hipError_t launch_records(const Launches& recs, hipStream_t s);

// ---- batched steps (many problems, one launch per kernel variant) ----

constexpr int kMaxRec = 32;  // launches of one step of one problem
// Stage slots of a variant: round (0: level 0's transpose, 1: the coarse
// transposes of an UNBIASED full-resolution sketch) times LDS class (the
// launches of one slot reserve the largest LDS among them, so launches that
// would fit different numbers of workgroups on a CU run in separate slots:
// the class bounds are 160 KB / k for k = 10, 8, 6, 5, 4, 3, 2).
constexpr int kLdsClasses = 8;
constexpr int kRounds = 2 * kLdsClasses;
inline int lds_class(int lds)
{
    constexpr int bound[kLdsClasses - 1] = {16 * 1024, 20 * 1024, 26 * 1024 + 682, 32 * 1024,
                                            40 * 1024, 53 * 1024 + 341, 80 * 1024};
    int c = 0;
    while (c < kLdsClasses - 1 && lds > bound[c]) ++c;
    return c;
}

// Per-problem counters, advanced on the device.  The sketch index of step k
// is drawn on the device from the same SplitMix64 stream as the host draw.
struct BatchProb {
    unsigned long long stream_state;  // SplitMix64 state of the problem's draw stream
    unsigned long long k;             // next draw
    unsigned long long k_stop;        // the problem idles from this draw on
    double epochs;
    int cur;
    int r;
    unsigned long long thr[IMASK_MAX_LEVELS];  // draw thresholds
    double cost[IMASK_MAX_LEVELS];             // epochs of each sketch
};

// One launch of one problem's step: which variant and round, its argument
// block and its grid (items = gx gy gz workgroups).
struct BatchRec {
    int variant, round, blob;
    int gx, gy, gz, items;
    int lds;  // dynamic LDS the launch needs
    int ord, ibefore;  // earlier records of this step with the same stage slot: count and items
};

// Device pointers of a batch buffer.
struct BatchView {
    int n, r_max;
    BatchProb* prob;         // n
    const BatchRec* rec;     // [n][r_max][2][kMaxRec]
    const int* nrec;         // [n][r_max][2]
    const int* items;        // [n][r_max][2][kNumVariants][kRounds]
    const unsigned char* blobs;  // argument blocks, kBlobBytes each
    int* off;                // [kNumVariants][kRounds][n + 1]: per-step item offsets
    int* sel;                // [n]: this step's (sketch index, parity) slot, -1 when idle
    const int* nsegs;        // [n][r_max][2][kNumVariants][kRounds]: records of each stage slot
    int* segc;               // [kNumVariants][kRounds][n + 1]: per-step record offsets per problem
    int* seg_off;            // [kNumVariants * kRounds + 1]: first segment of each stage slot
    int* seg;                // [n kMaxRec][2]: per-step (record index, first item) of each stage slot's records
    const int* rank;         // [n]: position of problem q in the work order (largest problems first)
};

int variant_threads(int v);
size_t variant_static_lds(int v);
hipError_t batch_allow_lds(int v, int lds);
hipError_t launch_batch_plan(const BatchView& bv, hipStream_t s);
hipError_t launch_batch_stage(int v, int round, const BatchView& bv, unsigned grid, int lds, hipStream_t s);
hipError_t launch_batch_advance(const BatchView& bv, hipStream_t s);

}  // namespace imk
