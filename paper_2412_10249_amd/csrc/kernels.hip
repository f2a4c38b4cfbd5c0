// kernels.hip - gfx950 kernels of the ImaSk hot path.
//
// Projector pair (Sec. 4.1, eq. (CT_sketches)): ray-driven Joseph forward
// projection R_l (k_fwd_band, k_fwd_direct) and a ray-driven transpose R_l^T
// (k_bp_own: every wavefront owns image rows in LDS, no atomics) that
// recomputes the forward's interpolation weights from the same 64-bit
// fixed-point coordinate, so the pair is an exact transpose.  Resampling
// (block mean T_l, compensation S_r) is done by the tile-pyramid kernel
// k_prep that feeds the projector; the SAGA table refresh and the primal /
// dual proximal steps of Alg. 1 are fused into the forward's reduce (dual)
// and into k_primal, or into the transpose's ordered partial sum when the
// sketch needs a single backprojection (k_bp_sum_primal); the smoothed-TV
// prox runs J FISTA iterations inside one launch on LDS-resident overlapped
// tiles (k_tv), the paper's TV prior J dual projected-gradient iterations
// (k_tvd).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"

namespace imk {

namespace {

// Default angles a*pi/na step along rows iff 4a <= na or 4a >= 3na; listed
// angles carry the host's choice (|cos| >= |sin|) in a table.
__device__ __forceinline__ bool row_stepping(int a, int na) { return 4 * a <= na || 4 * a >= 3 * na; }
__device__ __forceinline__ bool row_stepping(const AngleSplit& sp, int a, int na)
{
    return sp.rows ? sp.rows[a] != 0 : row_stepping(a, na);
}

constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// Left tap and right-tap weight of the fixed-point coordinate u.
__device__ __forceinline__ int tap_index(long long u) { return (int)(u >> 32); }
__device__ __forceinline__ float tap_weight(long long u) { return (float)(unsigned)(u & 0xffffffffLL) * kTwoM32; }

// Compiler-only ordering point between the two read-modify-write phases of
// a scatter (left taps, then right taps): LDS operations of one wavefront
// execute in program order, so keeping the compiler from moving them across
// is all that is needed.
#define IMK_LDS_ORDER() asm volatile("" ::: "memory")

// The block a kernel body works on: its grid coordinates and the grid's
// x extent (for grid-stride loops).  A kernel passes its own blockIdx; the
// batched kernels pass a block of one problem's launch taken from a work
// list, so the same body serves both.
struct Blk {
    int x, y, z, gx;
};
__device__ __forceinline__ Blk this_block()
{
    return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x};
}

// th / rows: listed angles (radians) and their stepping flags, or null for
// a*pi/na; side = 2E, the side of the image square.
__global__ void k_consts(int n, int na, int nd, double ds, double s0, double side, const double* th_tab,
                         const int* rows_tab, int lmax, RayConst* out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (lmax + 1) * na) return;
    const int l = idx / na, a = idx - l * na;
    const double th = th_tab ? th_tab[a] : (double)a * M_PI / (double)na;
    const bool rows = rows_tab ? rows_tab[a] != 0 : row_stepping(a, na);
    const double c = cos(th), s = sin(th);
    const int nl = n >> l;
    const double hl = side / nl;
    const double half = 0.5 * (nl - 1), halfd = 0.5 * (nd - 1);
    // u(i, b) = A (i - half) + B (b - halfd) + C, the column (row) coordinate
    // of ray b where it crosses row (column) i, in pixels of level l.
    double A, B, C, W;
    if (rows) {
        A = -s / c;
        B = ds / (hl * c);
        C = s0 / (hl * c) + half;
        W = hl / fabs(c);
    } else {
        A = -c / s;
        B = ds / (hl * s);
        C = s0 / (hl * s) + half;
        W = hl / fabs(s);
    }
    const double C0 = C - half * A - halfd * B;  // u(0, 0)
    const double scale = 4294967296.0;
    RayConst r;
    r.afx = __double2ll_rn(A * scale);
    r.bfx = __double2ll_rn(B * scale);
    r.cfx = __double2ll_rn(C0 * scale);
    const long long ab = r.bfx < 0 ? -r.bfx : r.bfx;
    r.phases = (int)((4294967296LL + ab - 1) / ab);
    r.pad = 0;
    r.a = (float)A;
    r.b = (float)B;
    r.c = (float)C0;
    r.w = (float)W;
    r.ib = (float)(1.0 / B);
    r.r0 = A != 0.0 ? (float)(1.0 / A) : 0.0f;  // 1/a, for step ranges without a division
    r.r1 = r.r2 = 0.0f;
    out[idx] = r;
}

__global__ void k_fill(float* p, size_t count, float value)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = i; q < count; q += stride) p[q] = value;
}

// ------------------------------------------------------------------ pyramid

// pyr holds a T x T tile at level 0 followed by its 2x2-mean levels.
__device__ __forceinline__ int pyr_offset(int T, int l)
{
    int off = 0;
    for (int q = 0; q < l; ++q) off += (T >> q) * (T >> q);
    return off;
}

__device__ void build_pyramid(float* pyr, int T, int levels)
{
    int off = 0, sd = T;
    for (int l = 0; l < levels; ++l) {
        const int ns = sd >> 1, noff = off + sd * sd;
        __syncthreads();
        for (int q = threadIdx.x; q < ns * ns; q += blockDim.x) {
            const int i = q / ns, j = q - i * ns;
            const float* s0 = pyr + off + (2 * i) * sd + 2 * j;
            pyr[noff + q] = 0.25f * ((s0[0] + s0[1]) + (s0[sd] + s0[sd + 1]));
        }
        off = noff;
        sd = ns;
    }
    __syncthreads();
}

__device__ __forceinline__ void load_tile(float* pyr, const float* x, int n, int T, int ty, int tx)
{
    for (int q = threadIdx.x; q < T * T; q += blockDim.x) {
        const int i = q / T, j = q - i * T;
        pyr[q] = x[(size_t)(ty * T + i) * n + tx * T + j];
    }
}

// Stores the outputs of one T x T tile (tile row ty, column tx) from its
// pyramid: block means at each output level, or the compensation S_r at
// level 0, into the padded row / transposed layouts of the projector.
__device__ __forceinline__ void prep_store(const PrepArgs& a, const float* pyr, int T, int ty, int tx)
{
    for (int o = 0; o < a.nout; ++o) {
        const PrepOut& po = a.out[o];
        const int l = po.lvl;
        const int tl = T >> l, nl = a.n >> l;
        const int P = po.padded ? nl + kPad : nl;
        const int sh = po.padded ? kPadL : 0;
        const int oy = ty * tl, ox = tx * tl;
        const int off = pyr_offset(T, l);
        for (int q = threadIdx.x; q < tl * tl; q += blockDim.x) {
            const int i = q / tl, j = q - i * tl;
            float v = pyr[off + q];
            if (po.kind == PREP_COMP) {
                float acc = v;
                for (int c = 0; c < a.ncomp; ++c) {
                    const int lc = a.comp_lvl[c];
                    const int tc = T >> lc;
                    acc -= a.comp_p[c] * pyr[pyr_offset(T, lc) + (i >> lc) * tc + (j >> lc)];
                }
                v = acc * a.inv_p0;
            }
            if (a.snap && a.snap_lvl == l && l > 0) {
                // compact tables, coarse sketch: T_l x - z_k, then z_k <- T_l x
                float* zc = a.snap + (size_t)(oy + i) * nl + ox + j;
                const float mean = v;
                v = mean - *zc;
                *zc = mean;
            }
            po.dst[(size_t)(oy + i) * P + ox + j + sh] = v;
            if (po.dstT) po.dstT[(size_t)(ox + j) * P + oy + i + sh] = v;
        }
    }
}

// Restricts (block mean at level l) or compensates (S_r at level 0) one
// T x T tile of x into padded row / transposed layouts for the projector.
__device__ __forceinline__ void prep_body(const PrepArgs& a, const Blk& bk, float* pyr)
{
    const int tiles = a.n / a.T;
    const int ty = bk.x / tiles, tx = bk.x - ty * tiles;
    if (a.snap && a.snap_lvl == 0) {
        // compact tables, full-resolution sketch: restrict x - z_0, then z_0 <- x
        for (int q = threadIdx.x; q < a.T * a.T; q += blockDim.x) {
            const int i = q / a.T, j = q - i * a.T;
            const size_t g = (size_t)(ty * a.T + i) * a.n + tx * a.T + j;
            const float xv = a.x[g];
            pyr[q] = xv - a.snap[g];
            a.snap[g] = xv;
        }
    } else {
        load_tile(pyr, a.x, a.n, a.T, ty, tx);
    }
    build_pyramid(pyr, a.T, a.pyr_levels);
    prep_store(a, pyr, a.T, ty, tx);
}

__global__ void __launch_bounds__(256) k_prep(PrepArgs a)
{
    extern __shared__ float pyr[];
    prep_body(a, this_block(), pyr);
}

// ---------------------------------------------------------- Joseph forward

__device__ __forceinline__ int angle_of(const AngleSplit& sp, int pass, int k)
{
    if (sp.perm) return sp.perm[pass == 0 ? k : sp.nrow + k];
    return pass == 0 ? (k < sp.n0a ? sp.s0a + k : sp.s0b + (k - sp.n0a)) : sp.s1 + k;
}

// Steps lo..hi (clamped to [s0, s1]) at which ray b's coordinate can reach
// [-1, nl]: a 0.01-pixel margin covers the float estimate, the zero padding
// of the image rows covers the rest.
__device__ __forceinline__ void ray_steps(const RayConst& kc, float fb, int nl, int s0, int s1, int& lo, int& hi)
{
    const float fnl = (float)nl;
    const float tf = fmaf(fb, kc.b, kc.c);  // ~coordinate at step 0
    lo = s0;
    hi = s1;
    if (kc.a != 0.0f) {
        // the reciprocal's relative error (~1e-7 of at most a few thousand
        // steps) is far inside the 0.01-pixel margin
        const float t1 = (-1.01f - tf) * kc.r0, t2 = (fnl + 0.01f - tf) * kc.r0;
        lo = (int)fminf(fmaxf(ceilf(fminf(t1, t2)), (float)s0), (float)(s1 + 1));
        hi = (int)fmaxf(fminf(floorf(fmaxf(t1, t2)), (float)s1), (float)(s0 - 1));
    } else if (tf < -1.01f || tf > fnl + 0.01f) {
        lo = s0 + 1;
        hi = s0;
    }
}

// Sum over steps lo..hi of the interpolated row values; rows are P floats
// apart starting at `row` (already offset by kPadL).
__device__ __forceinline__ float joseph_sum(const float* row, int P, long long u, long long du, int n)
{
    float acc = 0.0f;
    int i = 0;
    for (; i + 4 <= n; i += 4) {  // all eight taps are loaded before use
        const long long u1 = u + du, u2 = u1 + du, u3 = u2 + du;
        const float* p0 = row + tap_index(u);
        const float* p1 = row + P + tap_index(u1);
        const float* p2 = row + 2 * P + tap_index(u2);
        const float* p3 = row + 3 * P + tap_index(u3);
        const float a0 = p0[0], b0 = p0[1], a1 = p1[0], b1 = p1[1];
        const float a2 = p2[0], b2 = p2[1], a3 = p3[0], b3 = p3[1];
        const float w0 = tap_weight(u), w1 = tap_weight(u1), w2 = tap_weight(u2), w3 = tap_weight(u3);
        acc = fmaf(1.0f - w0, a0, acc);
        acc = fmaf(w0, b0, acc);
        acc = fmaf(1.0f - w1, a1, acc);
        acc = fmaf(w1, b1, acc);
        acc = fmaf(1.0f - w2, a2, acc);
        acc = fmaf(w2, b2, acc);
        acc = fmaf(1.0f - w3, a3, acc);
        acc = fmaf(w3, b3, acc);
        u = u3 + du;
        row += 4 * P;
    }
    for (; i < n; ++i) {
        const float* px = row + tap_index(u);
        const float w = tap_weight(u);
        acc = fmaf(1.0f - w, px[0], acc);
        acc = fmaf(w, px[1], acc);
        u += du;
        row += P;
    }
    return acc;
}

// Sum along one ray over a band held in LDS.  U's high word is the LDS cell
// of the left tap (the row offset folded in), dU advances one row.  The
// interpolation (1-w) a + w b is accumulated as sum(a) + 2^-32 sum(f (b - a))
// with f = 2^32 w the coordinate's low word: four VALU operations per sample
// besides the coordinate step and the address.  A single term reproduces the
// transpose's matrix entries exactly (1-w rounded once, w exact).
__device__ __forceinline__ float band_sum(const float* band, long long U, long long dU, int n)
{
    float s1 = 0.0f, s2 = 0.0f;
    int i = 0;
    // four coordinates a row apart, each advanced by four rows per trip
    long long u1 = U + dU, u2 = U + 2 * dU, u3 = U + 3 * dU;
    const long long d4 = 4 * dU;
    for (; i + 4 <= n; i += 4) {  // all eight taps are loaded before use
        const float* p0 = band + (int)(U >> 32);
        const float* p1 = band + (int)(u1 >> 32);
        const float* p2 = band + (int)(u2 >> 32);
        const float* p3 = band + (int)(u3 >> 32);
        const float a0 = p0[0], b0 = p0[1], a1 = p1[0], b1 = p1[1];
        const float a2 = p2[0], b2 = p2[1], a3 = p3[0], b3 = p3[1];
        s1 += a0;
        s2 = fmaf((float)(unsigned)(U & 0xffffffffLL), b0 - a0, s2);
        s1 += a1;
        s2 = fmaf((float)(unsigned)(u1 & 0xffffffffLL), b1 - a1, s2);
        s1 += a2;
        s2 = fmaf((float)(unsigned)(u2 & 0xffffffffLL), b2 - a2, s2);
        s1 += a3;
        s2 = fmaf((float)(unsigned)(u3 & 0xffffffffLL), b3 - a3, s2);
        U += d4;
        u1 += d4;
        u2 += d4;
        u3 += d4;
        // opaque to induction-variable rewriting: keeps one 64-bit add per coordinate
        asm("" : "+v"(U), "+v"(u1), "+v"(u2), "+v"(u3));
    }
    for (; i < n; ++i) {
        const float* p = band + (int)(U >> 32);
        const float a0 = p[0], b0 = p[1];
        s1 += a0;
        s2 = fmaf((float)(unsigned)(U & 0xffffffffLL), b0 - a0, s2);
        U += dU;
    }
    return fmaf(s2, kTwoM32, s1);
}

// LDS-band forward: the workgroup copies rows [i0, i0+R) of the padded level
// image (columns of it for column-stepping angles) into LDS and sums, for
// every ray of its angle group, the samples falling in the band.  The ray's
// partial sum goes to part[band][a][b]; k_fwd_reduce adds the bands in order.
__device__ __forceinline__ void fwd_band_body(const FwdBandArgs& a, const Blk& bk, float* band)
{
    const int nl = a.n >> a.lvl;
    const int P = nl + kPad;
    const int bi = bk.x;    // band
    const int gidx = bk.y;  // angle group (row-stepping groups first)
    const int pass = gidx < a.groups_row ? 0 : 1;
    const int g = pass == 0 ? gidx : gidx - a.groups_row;
    const int npass = pass == 0 ? a.split.nrow : a.split.ncol;
    // group g of its pass takes angles g, g + G, g + 2G, ...: every workgroup
    // gets the same mix of steep and shallow angles (a ray's sample count
    // follows max(|cos|, |sin|)), so no group is left running alone at the end
    const int G = pass == 0 ? a.groups_row : a.groups_col;
    const int nang = (npass - g + G - 1) / G;
    const int i0 = bi * a.R;
    const int i1 = min(nl, i0 + a.R);
    {
        const float* src = (pass == 0 ? a.img : a.imgT) + (size_t)i0 * P;
        const int cnt = (i1 - i0) * P;
        if ((P & 3) == 0) {  // rows start 16-byte aligned
            const float4* s4 = (const float4*)src;
            float4* d4 = (float4*)band;
            for (int q = threadIdx.x; q < cnt / 4; q += blockDim.x) d4[q] = s4[q];
        } else {
            for (int q = threadIdx.x; q < cnt; q += blockDim.x) band[q] = src[q];
        }
    }
    __syncthreads();
    const size_t m = (size_t)a.na * a.nd;
    const long long rowfx = (long long)P << 32;
    // (angle kk, bin b) of this thread's ray, advanced without a division
    int kk = threadIdx.x / a.nd;
    int b = threadIdx.x - kk * a.nd;
    while (kk < nang) {
        const int ang = angle_of(a.split, pass, g + kk * G);
        const RayConst& kc = a.consts[(size_t)a.lvl * a.na + ang];
        int lo, hi;
        ray_steps(kc, (float)b, nl, i0, i1 - 1, lo, hi);
        float acc = 0.0f;
        if (lo <= hi) {
            const long long U = kc.cfx + (long long)b * kc.bfx + (long long)lo * kc.afx +
                                (long long)((lo - i0) * P + kPadL) * 4294967296LL;
            acc = band_sum(band, U, kc.afx + rowfx, hi - lo + 1);
        }
        const float total = kc.w * acc;
        if (a.dual) {
            // the reduce's dual step for this ray: zeta = psi_new - psi_k +
            // sum_j p_j psi_j (old tables), y+ = (y + sigma zeta - sigma b)/(1 + sigma)
            const size_t e = (size_t)ang * a.nd + b;
            float avg = 0.0f;
            for (int j = 0; j < a.r; ++j) avg = fmaf(a.p[j], a.psi[(size_t)j * m + e], avg);
            float* pk = a.psi + (size_t)a.kidx * m + e;
            const float zeta = (total - *pk) + avg;
            a.y_new[e] = (a.y_old[e] + a.sigma * zeta - a.sigma * a.bdat[e]) * a.inv1ps;
            *pk = total;
        } else {
            a.part[(size_t)bi * m + (size_t)ang * a.nd + b] = total;
        }
        b += blockDim.x;
        while (b >= a.nd) {
            b -= a.nd;
            ++kk;
        }
    }
}

__global__ void __launch_bounds__(1024) k_fwd_band(FwdBandArgs a)
{
    extern __shared__ float band[];
    fwd_band_body(a, this_block(), band);
}

// Direct forward for levels too large for LDS bands: one thread per ray
// reading the padded image from global memory; writes a single band.
__device__ __forceinline__ void fwd_direct_body(const FwdBandArgs& a, const Blk& bk)
{
    const int lane = threadIdx.x & 63;
    const int wpa = (a.nd + 63) >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(bk.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int ang = __builtin_amdgcn_readfirstlane(wave / wpa);
    if (ang >= a.na) return;
    const int b = (wave - ang * wpa) * 64 + lane;
    if (b >= a.nd) return;
    const int nl = a.n >> a.lvl;
    const int P = nl + kPad;
    const RayConst& kc = a.consts[(size_t)a.lvl * a.na + ang];
    const float* img = row_stepping(a.split, ang, a.na) ? a.img : a.imgT;
    int lo, hi;
    ray_steps(kc, (float)b, nl, 0, nl - 1, lo, hi);
    float acc = 0.0f;
    if (lo <= hi) {
        const long long u = kc.cfx + (long long)b * kc.bfx + (long long)lo * kc.afx;
        acc = joseph_sum(img + (size_t)lo * P + kPadL, P, u, kc.afx, hi - lo + 1);
    }
    a.part[(size_t)ang * a.nd + b] = kc.w * acc;
}

__global__ void __launch_bounds__(256) k_fwd_direct(FwdBandArgs a) { fwd_direct_body(a, this_block()); }

// ------------------------------------------------------------ fan beam

// Fixed-point Joseph coordinate of fan ray r on a level of nl pixels per
// side: u(step) = cfx + step * afx in units of 2^-32 pixel (high word the
// left tap, low word the right tap's weight), and the step length w.  Both
// kernels of the fan pair call this; the explicit fma leaves the compiler
// no multiply-add to fuse differently in the two, so they agree on every
// weight bit for bit.
__device__ __forceinline__ void fan_coords(const FanRay& r, double E, int nl, long long& cfx, long long& afx,
                                           float& w)
{
    const double hl = 2.0 * E / nl;
    const double C = fma(E - 0.5 * hl, r.T + 1.0, r.P) * ((double)nl / (2.0 * E));
    cfx = __double2ll_rn(C * 4294967296.0);
    afx = __double2ll_rn(-r.T * 4294967296.0);
    w = (float)(hl * r.sec);
}

// Fan-beam forward: one thread per ray walks every row (row-stepping rays)
// or column (column-stepping rays, on the transposed copy) of the padded
// level image and interpolates between the two taps; taps outside the image
// read the zero padding, and steps whose taps both lie outside are skipped.
__global__ void __launch_bounds__(256) k_fwd_fan(FwdBandArgs a)
{
    const size_t e = (size_t)a.fan.va * a.nd + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = e < (size_t)a.fan.vb * a.nd;  // lanes past the end still take part in the range vote
    const int nl = a.n >> a.lvl;
    const int P = nl + kPad;
    FanRay r{};
    long long cfx = 0, afx = 0;
    float wr = 0.0f;
    // the steps whose left tap can lie in [-1, nl - 1], from the line
    // u(k) = cfx + k afx in FP64, one step wider on each side (empty past
    // the end); the wavefront walks the union of its lanes' ranges, so its
    // loads at a step stay on one row, and the exact test below decides
    // every step: the sum is the full walk's, bit for bit
    int k0 = nl, k1 = -1;
    if (ok) {
        r = a.fan.ray[e];
        fan_coords(r, a.fan.E, nl, cfx, afx, wr);
        if (afx != 0) {
            const double t1 = (-4294967296.0 - (double)cfx) / (double)afx;
            const double t2 = ((double)nl * 4294967296.0 - (double)cfx) / (double)afx;
            k0 = (int)fmin(fmax(floor(fmin(t1, t2)) - 1.0, 0.0), (double)nl);
            k1 = (int)fmax(fmin(ceil(fmax(t1, t2)) + 1.0, (double)(nl - 1)), -1.0);
        } else {
            k0 = 0;
            k1 = nl - 1;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        k0 = min(k0, __shfl_xor(k0, off));
        k1 = max(k1, __shfl_xor(k1, off));
    }
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
    const float* img = (r.row ? a.img : a.imgT) + kPadL;
    float acc = 0.0f;
    long long u = cfx + (long long)k0 * afx;
    for (int k = k0; k <= k1; ++k, u += afx) {
        const int j0 = tap_index(u);
        if (ok && (unsigned)(j0 + 1) <= (unsigned)nl) {  // j0 in [-1, nl - 1]
            const float w = tap_weight(u);
            const float* t = img + (size_t)k * P + j0;
            acc = fmaf(1.0f - w, t[0], fmaf(w, t[1], acc));
        }
    }
    if (ok) a.part[e] = wr * acc;
}

// Fan-beam forward over LDS bands, as k_fwd_band for the parallel beam:
// workgroup (band, group) copies rows [i0, i1) of the padded level image
// (pass 0) or of its transposed copy (pass 1) into LDS, and sums over the
// band every ray of its views that steps along that axis; each ray's line
// is its own (the ray table's fixed-point coordinate), its steps in the
// band come from that line in FP64, one step wider on each side (a tap one
// step outside the image lands in the zero padding and adds nothing).
// View group g of a pass takes the views va + g, va + g + G, ...  The ray's
// band sum goes to part[band][view][bin]; the reduce adds the bands.
__global__ void __launch_bounds__(1024) k_fwd_fan_band(FwdBandArgs a)
{
    extern __shared__ float band[];
    const int nl = a.n >> a.lvl;
    const int P = nl + kPad;
    const int bi = blockIdx.x;
    const int G = a.groups_row;  // view groups per pass
    const int pass = (int)blockIdx.y < G ? 0 : 1;
    const int g = (int)blockIdx.y - pass * G;
    const FanGeo& f = a.fan;
    const int nv = f.vb - f.va;
    const int nvg = g < nv ? (nv - g + G - 1) / G : 0;
    const int i0 = bi * a.R;
    const int i1 = min(nl, i0 + a.R);
    {
        const float* src = (pass == 0 ? a.img : a.imgT) + (size_t)i0 * P;
        const int cnt = (i1 - i0) * P;
        if ((P & 3) == 0) {  // rows start 16-byte aligned
            const float4* s4 = (const float4*)src;
            float4* d4 = (float4*)band;
            for (int q = threadIdx.x; q < cnt / 4; q += blockDim.x) d4[q] = s4[q];
        } else {
            for (int q = threadIdx.x; q < cnt; q += blockDim.x) band[q] = src[q];
        }
    }
    __syncthreads();
    const size_t m = (size_t)a.na * a.nd;
    const long long rowfx = (long long)P << 32;
    int kk = threadIdx.x / a.nd;
    int b = threadIdx.x - kk * a.nd;
    while (kk < nvg) {
        const size_t e = (size_t)(f.va + g + kk * G) * a.nd + b;
        const FanRay r = f.ray[e];
        if ((r.row != 0) == (pass == 0)) {
            long long cfx, afx;
            float wr;
            fan_coords(r, f.E, nl, cfx, afx, wr);
            int lo = i0, hi = i1 - 1;
            if (afx != 0) {
                const double t1 = (-4294967296.0 - (double)cfx) / (double)afx;
                const double t2 = ((double)nl * 4294967296.0 - (double)cfx) / (double)afx;
                lo = (int)fmin(fmax(floor(fmin(t1, t2)) - 1.0, (double)i0), (double)i1);
                hi = (int)fmax(fmin(ceil(fmax(t1, t2)) + 1.0, (double)(i1 - 1)), (double)(i0 - 1));
            } else if ((unsigned)((int)(cfx >> 32) + 1) > (unsigned)nl) {
                lo = i0 + 1;  // a line outside the image: no step
                hi = i0;
            }
            float acc = 0.0f;
            if (lo <= hi) {
                const long long U = cfx + (long long)lo * afx + (long long)((lo - i0) * P + kPadL) * 4294967296LL;
                acc = band_sum(band, U, afx + rowfx, hi - lo + 1);
            }
            a.part[(size_t)bi * m + e] = wr * acc;
        }
        b += blockDim.x;
        while (b >= a.nd) {
            b -= a.nd;
            ++kk;
        }
    }
}

// Fan-beam transpose as a gather, for levels where rays are dense (more than
// kFanScatterMaxP phases of the scatter below): 16 x 16 pixel tiles, one
// workgroup per tile and view group.  In a view, the row-stepping rays that
// put a tap on pixel (i, j) are those crossing its row between the centres
// of pixels j - 1 and j + 1 (column-stepping ones: its column between rows
// i - 1 and i + 1); those end points, projected from the source onto the
// detector, bound the pixel's candidate bins, and the projections of the
// tile's two end-point boxes bound the tile's.  Each round stages the
// tile's candidate bins of the next kFanViews views of the group (at most
// kFanSlots bins; a view with more continues in the next round) through
// LDS, each bin with the forward's fixed-point coordinate and its weighted
// datum; every pixel then tests its own candidates exactly and adds (1 - w)
// or w of the datum, so every matrix entry is the forward's bit for bit.
// Bin estimates are FP32 with a margin (bmargin) well above their rounding
// error: a spare candidate fails the exact test, none is missed.  A pixel
// sums its rays in the group's view order and bin order, row-stepping
// candidates before column-stepping ones within a staged segment of a view.
constexpr int kFanTile = 16;
constexpr int kFanSlots = 512;
#ifndef IMK_FAN_TARGET_WG
#define IMK_FAN_TARGET_WG 8192
#endif
constexpr int kFanViews = 16;

__global__ void __launch_bounds__(256) k_bp_fan_gather(BpOwnArgs a)
{
    __shared__ long long s_cfx[kFanSlots], s_afx[kFanSlots];
    __shared__ float s_wy[kFanSlots];
    __shared__ int s_row[kFanSlots];
    __shared__ int q_lo[kFanViews], q_hi[kFanViews], q_fl[kFanViews];  // the round's views: tile ranges, axes
    __shared__ float q_c[kFanViews], q_s[kFanViews];
    __shared__ int g_view[kFanViews + 1], g_b0[kFanViews + 1], g_start[kFanViews + 1];  // segments
    __shared__ int g_n, g_next_v, g_next_b;
    const int nl = a.n >> a.lvl;
    const int tiles = (nl + kFanTile - 1) / kFanTile;
    const int ty = blockIdx.x / tiles, tx = blockIdx.x - ty * tiles;
    const int i = ty * kFanTile + (threadIdx.x >> 4), j = tx * kFanTile + (threadIdx.x & 15);
    const bool inside = i < nl && j < nl;
    const int g = blockIdx.y;
    const FanGeo& f = a.fan;
    // group g takes the views va + g, va + g + G, ... (the same mix of view
    // angles in every group); v below counts the group's views
    const int nvg = g < f.vb - f.va ? (f.vb - f.va - g + a.G - 1) / a.G : 0;
    auto view_of = [&](int k) { return f.va + g + k * a.G; };
    const double hl = 2.0 * f.E / nl;
    auto ctr = [&](int k) { return (float)(-f.E + (k + 0.5) * hl); };  // pixel-centre coordinate
    const float xj = ctr(j), yi = ctr(i), hf = (float)hl;
    const float Df = (float)f.D, mag = (float)(f.D + f.Dd), ids = (float)(1.0 / f.ds);
    const float bofs = (float)(0.5 * (a.nd - 1) - f.s0 / f.ds), marg = f.bmargin, top = (float)(a.nd - 1);
    // detector bin coordinate of a point seen from the source of view (c, s)
    auto bin = [&](float c, float s, float x, float y) {
        return mag * (c * y - s * x) * __builtin_amdgcn_rcpf(Df - (c * x + s * y)) * ids + bofs;
    };
    // a bin interval's first and last candidates, clamped before the conversion
    auto first = [&](float lo) { return (int)ceilf(fminf(fmaxf(lo - marg, 0.0f), top + 1.0f)); };
    auto last = [&](float hi) { return (int)floorf(fmaxf(fminf(hi + marg, top), -1.0f)); };
    float acc = 0.0f;
    int v = 0, boff = -1;  // next view; first bin still to stage in it (-1: its tile range start)
    while (v < nvg) {
        __syncthreads();  // the previous round's LDS has been read
        if ((int)threadIdx.x < kFanViews) {
            // tile range of view v + t: projections of the end-point boxes
            // (row pass: x over centres tx*16-1 .. tx*16+16, y over the tile's
            // rows; column pass the mirror), all within 1.6E of the centre
            const int t = threadIdx.x, vv = v + t;
            int lo = 0, hi = -1, fl = 0;
            float c = 0.0f, s = 0.0f;
            if (vv < nvg) {
                const FanView fv = f.view[view_of(vv)];
                c = (float)fv.c;
                s = (float)fv.s;
                fl = (fv.has_row ? 1 : 0) | (fv.has_col ? 2 : 0);
                const int e0 = tx * kFanTile, e1 = min(e0 + kFanTile, nl);
                const int r0 = ty * kFanTile, r1 = min(r0 + kFanTile, nl);
                float blo = 3.0e38f, bhi = -3.0e38f;
                auto box = [&](float x0, float x1, float y0, float y1) {
                    const float q0 = bin(c, s, x0, y0), q1 = bin(c, s, x1, y0);
                    const float q2 = bin(c, s, x0, y1), q3 = bin(c, s, x1, y1);
                    blo = fminf(blo, fminf(fminf(q0, q1), fminf(q2, q3)));
                    bhi = fmaxf(bhi, fmaxf(fmaxf(q0, q1), fmaxf(q2, q3)));
                };
                if (fl & 1) box(ctr(e0 - 1), ctr(e1), ctr(r0), ctr(r1 - 1));
                if (fl & 2) box(ctr(e0), ctr(e1 - 1), ctr(r0 - 1), ctr(r1));
                lo = first(blo);
                hi = last(bhi);
            }
            q_lo[t] = lo;
            q_hi[t] = hi;
            q_fl[t] = fl;
            q_c[t] = c;
            q_s[t] = s;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // cut the round into segments of the views' ranges, kFanSlots bins in all
            int n = 0, used = 0, nv = v, nb = -1;
            for (int k = 0; k < kFanViews && v + k < nvg; ++k) {
                const int lo = (k == 0 && boff >= 0) ? boff : q_lo[k];
                const int cnt = q_hi[k] - lo + 1;
                const int take = min(cnt, kFanSlots - used);
                if (take > 0) {
                    g_view[n] = k;
                    g_b0[n] = lo;
                    g_start[n] = used;
                    ++n;
                    used += take;
                }
                if (take < cnt) {  // the view continues next round
                    nv = v + k;
                    nb = lo + take;
                    break;
                }
                nv = v + k + 1;
            }
            g_start[n] = used;
            g_n = n;
            g_next_v = nv;
            g_next_b = nb;
        }
        __syncthreads();
        const int n = g_n, used = g_start[n];
        for (int sl = threadIdx.x; sl < used; sl += blockDim.x) {
            int k = 0;
            while (k + 1 < n && g_start[k + 1] <= sl) ++k;
            const int vv = view_of(v + g_view[k]), b = g_b0[k] + (sl - g_start[k]);
            const FanRay r = f.ray[(size_t)vv * a.nd + b];
            long long cfx, afx;
            float wr;
            fan_coords(r, f.E, nl, cfx, afx, wr);
            s_cfx[sl] = cfx;
            s_afx[sl] = afx;
            s_wy[sl] = wr * a.y[(size_t)vv * a.nd + b];
            s_row[sl] = r.row;
        }
        const int next_v = g_next_v, next_b = g_next_b;
        __syncthreads();
        if (inside) {
            for (int k = 0; k < n; ++k) {
                const int kv = g_view[k], fl = q_fl[kv];
                const float c = q_c[kv], s = q_s[kv];
                const int b0 = g_b0[k], b1 = b0 + (g_start[k + 1] - g_start[k]) - 1, base = g_start[k] - b0;
                if (fl & 1) {
                    const float p0 = bin(c, s, xj - hf, yi), p1 = bin(c, s, xj + hf, yi);
                    const int lo = max(b0, first(fminf(p0, p1))), hi = min(b1, last(fmaxf(p0, p1)));
                    for (int b = lo; b <= hi; ++b) {
                        const int sl = b + base;
                        if (!s_row[sl]) continue;
                        const long long u = s_cfx[sl] + (long long)i * s_afx[sl];
                        const int t = tap_index(u);
                        if (t == j)
                            acc = fmaf(1.0f - tap_weight(u), s_wy[sl], acc);
                        else if (t == j - 1)
                            acc = fmaf(tap_weight(u), s_wy[sl], acc);
                    }
                }
                if (fl & 2) {
                    const float p0 = bin(c, s, xj, yi - hf), p1 = bin(c, s, xj, yi + hf);
                    const int lo = max(b0, first(fminf(p0, p1))), hi = min(b1, last(fmaxf(p0, p1)));
                    for (int b = lo; b <= hi; ++b) {
                        const int sl = b + base;
                        if (s_row[sl]) continue;
                        const long long u = s_cfx[sl] + (long long)j * s_afx[sl];
                        const int t = tap_index(u);
                        if (t == i)
                            acc = fmaf(1.0f - tap_weight(u), s_wy[sl], acc);
                        else if (t == i - 1)
                            acc = fmaf(tap_weight(u), s_wy[sl], acc);
                    }
                }
            }
        }
        v = next_v;
        boff = next_b;
    }
    if (inside) a.part[(size_t)g * nl * nl + (size_t)i * nl + j] = acc;
}

// Per-launch table of the fan transpose: every ray's fixed-point
// coordinate on this level (fan_coords, as the forward computes it) and its
// weighted datum w_ray * y.
__global__ void __launch_bounds__(256) k_fan_table(BpOwnArgs a)
{
    const size_t e = (size_t)a.fan.va * a.nd + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)a.fan.vb * a.nd) return;
    const int nl = a.n >> a.lvl;
    const FanRay r = a.fan.ray[e];
    FanTab t;
    float wr;
    fan_coords(r, a.fan.E, nl, t.cfx, t.afx, wr);
    t.wy = wr * a.y[e];
    t.row = r.row;
    a.fan.tab[e] = t;
}

// Fan-beam transpose as an ownership scatter.  Workgroup (block, pass,
// group) owns RW * waves image rows (pass 0, row-stepping rays) or columns
// (pass 1, column-stepping rays) in LDS, RW per wavefront, each with one
// cell beyond either end of the image for the taps that fall outside it.
// A wavefront reads each ray's table entry once for all its RW lines.
// For each view of its group, every wavefront takes the bins that can reach
// the block (the projection of the block's end-point box, FP32 with a
// margin) in P phases: lanes of one instruction hold bins P apart, and P is
// chosen so that such rays are more than a pixel apart at every owned cell,
// so no two lanes of an instruction update the same cell.  A lane takes CH
// rays per trip, 64 P bins apart (every ray of a trip is at least P bins
// from every other), and issues all their cells' reads before the writes,
// so the LDS latencies overlap.  A sample adds (1 - w) of its ray's
// weighted datum to the left tap, then w to the right tap: the forward's
// weights bit for bit, in a fixed order.  Used where P <= kFanScatterMaxP.
#ifndef IMK_FAN_ROWS_SPARSE
#define IMK_FAN_ROWS_SPARSE 3
#endif
#ifndef IMK_FAN_ROWS_DENSE
#define IMK_FAN_ROWS_DENSE 4
#endif
#ifndef IMK_FAN_SPARSE_WAVES
#define IMK_FAN_SPARSE_WAVES 4
#endif
constexpr int kFanMaxWaves = 8;
#ifndef IMK_FAN_SCATTER_MAX_P
#define IMK_FAN_SCATTER_MAX_P 6
#endif
constexpr int kFanScatterMaxP = IMK_FAN_SCATTER_MAX_P;
#ifndef IMK_FAN_SCATTER_WG
#define IMK_FAN_SCATTER_WG 4096
#endif

template <int CH, int RW>
__global__ void __launch_bounds__(kFanMaxWaves * 64) k_bp_fan_scatter(BpOwnArgs a, int P)
{
    extern __shared__ float cells[];  // owned lines of nl + 2 cells: taps -1 .. nl
    const int nl = a.n >> a.lvl;
    const int S = nl + 2;
    const int rows = RW * (int)(blockDim.x >> 6);
    const int pass = blockIdx.y, g = blockIdx.z;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q0 = blockIdx.x * rows;  // first owned row (pass 0) or column (pass 1)
    const int nown = min(rows, nl - q0);
    for (int c = threadIdx.x; c < rows * S; c += blockDim.x) cells[c] = 0.0f;
    __syncthreads();
    const FanGeo& f = a.fan;
    // group g takes the views va + g, va + g + G, ...: every group sees the
    // same mix of view angles, so the row and column passes' workgroups get
    // about equal work
    const int nvg = g < f.vb - f.va ? (f.vb - f.va - g + a.G - 1) / a.G : 0;
    const double hl = 2.0 * f.E / nl;
    auto ctr = [&](int k) { return (float)(-f.E + (k + 0.5) * hl); };  // pixel-centre coordinate
    const float Df = (float)f.D, mag = (float)(f.D + f.Dd), ids = (float)(1.0 / f.ds);
    const float bofs = (float)(0.5 * (a.nd - 1) - f.s0 / f.ds), marg = f.bmargin, top = (float)(a.nd - 1);
    // the block's end-point box: its own lines' centres along the owned
    // axis, the centres -1 .. nl across it (all within 1.6E of the centre)
    const float o0 = ctr(q0), o1 = ctr(q0 + nown - 1), x0 = ctr(-1), x1 = ctr(nl);
    const int want = pass == 0 ? 1 : 0;
    for (int jv = 0; jv < nvg; ++jv) {
        const int v = f.va + g + jv * a.G;
        const FanView fv = f.view[v];
        if (pass == 0 ? !fv.has_row : !fv.has_col) continue;
        const float c = (float)fv.c, s = (float)fv.s;
        auto bin = [&](float x, float y) {
            return mag * (c * y - s * x) * __builtin_amdgcn_rcpf(Df - (c * x + s * y)) * ids + bofs;
        };
        float q[4];
        if (pass == 0) {
            q[0] = bin(x0, o0);
            q[1] = bin(x1, o0);
            q[2] = bin(x0, o1);
            q[3] = bin(x1, o1);
        } else {
            q[0] = bin(o0, x0);
            q[1] = bin(o0, x1);
            q[2] = bin(o1, x0);
            q[3] = bin(o1, x1);
        }
        const float lo = fminf(fminf(q[0], q[1]), fminf(q[2], q[3]));
        const float hi = fmaxf(fmaxf(q[0], q[1]), fmaxf(q[2], q[3]));
        const int blo = (int)ceilf(fminf(fmaxf(lo - marg, 0.0f), top + 1.0f));
        const int bhi = (int)floorf(fmaxf(fminf(hi + marg, top), -1.0f));
        const FanTab* tv = f.tab + (size_t)v * a.nd;
        for (int p = 0; p < P; ++p) {
            for (int b = blo + p + P * lane; b <= bhi; b += CH * 64 * P) {
                constexpr int NC = CH * RW;
                int cl[NC];
                bool ok[NC];
                float omw[NC], cw[NC], wy[NC];
#pragma unroll
                for (int h = 0; h < CH; ++h) {
                    const int bh = b + h * 64 * P;
                    FanTab t{};
                    if (bh <= bhi) t = tv[bh];
                    const bool use = bh <= bhi && t.row == want;
#pragma unroll
                    for (int rr = 0; rr < RW; ++rr) {
                        const int c = h * RW + rr;
                        const int own = wave * RW + rr;
                        const long long u = t.cfx + (long long)(q0 + own) * t.afx;
                        const int j0 = tap_index(u);
                        ok[c] = use && own < nown && (unsigned)(j0 + 1) <= (unsigned)nl;  // j0 in [-1, nl - 1]
                        cl[c] = own * S + 1 + (ok[c] ? j0 : 0);
                        cw[c] = tap_weight(u);
                        omw[c] = 1.0f - cw[c];
                        wy[c] = t.wy;
                    }
                }
                float old[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) old[c] = ok[c] ? cells[cl[c]] : 0.0f;
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    if (ok[c]) cells[cl[c]] = fmaf(omw[c], wy[c], old[c]);
                IMK_LDS_ORDER();
#pragma unroll
                for (int c = 0; c < NC; ++c) old[c] = ok[c] ? cells[cl[c] + 1] : 0.0f;
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    if (ok[c]) cells[cl[c] + 1] = fmaf(cw[c], wy[c], old[c]);
                IMK_LDS_ORDER();
            }
        }
    }
    __syncthreads();
    // owned rows into partial image 2g, owned columns into 2g + 1
    float* out = a.part + (size_t)(2 * g + pass) * nl * nl;
    if (pass == 0) {
        for (int e = threadIdx.x; e < nown * nl; e += blockDim.x) {
            const int r = e / nl, j = e - r * nl;
            out[(size_t)(q0 + r) * nl + j] = cells[r * S + 1 + j];
        }
    } else {
        for (int e = threadIdx.x; e < nl * nown; e += blockDim.x) {
            const int i = e / nown, k = e - i * nown;
            out[(size_t)i * nl + q0 + k] = cells[k * S + 1 + i];
        }
    }
}

// Adds the band partials of every term (in band order), then stores,
// accumulates, or applies the dual SAGA step of Alg. 1:
// zeta = psi_new - psi_k + sum_j p_j psi_j (old tables),
// y+ = (y + sigma zeta - sigma b)/(1 + sigma), psi_k <- psi_new.
__device__ __forceinline__ void fwd_reduce_body(const FwdArgs& a, const Blk& bk)
{
    const size_t m = (size_t)a.na * a.nd;
    for (size_t e = (size_t)bk.x * blockDim.x + threadIdx.x; e < m; e += (size_t)bk.gx * blockDim.x) {
        float total = 0.0f;
        for (int t = 0; t < a.nterms; ++t) {
            const float* pp = a.term[t].part + e;
            float sum = 0.0f;
            for (int bnd = 0; bnd < a.term[t].bands; ++bnd) sum += pp[(size_t)bnd * m];
            total = fmaf(a.term[t].coef, sum, total);
        }
        if (a.mode == FWD_STORE) {
            a.out[e] = total;
        } else if (a.mode == FWD_ACCUM) {
            a.out[e] += total;
        } else if (a.compact) {
            // total = K_k (x - z_k) = psi_new - psi_k; psi holds the average
            const float avg = a.psi[e];
            const float zeta = total + avg;
            a.y_new[e] = (a.y_old[e] + a.sigma * zeta - a.sigma * a.bdat[e]) * a.inv1ps;
            a.psi[e] = fmaf(a.p[a.kidx], total, avg);
        } else {
            // outside this step's measurement block the sketch is zero and
            // so is its table: zeta is the table average alone
            const bool in = (long long)e >= a.e0 && (long long)e < a.e1;
            float avg = 0.0f;
            for (int j = 0; j < a.r; ++j) avg = fmaf(a.p[j], a.psi[(size_t)j * m + e], avg);
            const float zeta = in ? (total - a.psi[(size_t)a.kidx * m + e]) + avg : avg;
            a.y_new[e] = (a.y_old[e] + a.sigma * zeta - a.sigma * a.bdat[e]) * a.inv1ps;
            if (in) a.psi[(size_t)a.kidx * m + e] = total;
        }
    }
}

__global__ void __launch_bounds__(256) k_fwd_reduce(FwdArgs a) { fwd_reduce_body(a, this_block()); }

// k_fwd_reduce on four consecutive elements per thread with 16-byte loads
// and stores (sinogram size a multiple of 4): the same arithmetic per element.
__device__ __forceinline__ void ld4(const float* p, float* v)
{
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}
__device__ __forceinline__ void st4(float* p, const float* v)
{
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ void fwd_reduce4_body(const FwdArgs& a, const Blk& bk)
{
    const size_t m = (size_t)a.na * a.nd;
    for (size_t e = ((size_t)bk.x * blockDim.x + threadIdx.x) * 4; e < m; e += (size_t)bk.gx * blockDim.x * 4) {
        float total[4] = {0.0f, 0.0f, 0.0f, 0.0f}, v[4];
        for (int t = 0; t < a.nterms; ++t) {
            const float* pp = a.term[t].part + e;
            float sum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int bnd = 0; bnd < a.term[t].bands; ++bnd) {
                ld4(pp + (size_t)bnd * m, v);
#pragma unroll
                for (int c = 0; c < 4; ++c) sum[c] += v[c];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) total[c] = fmaf(a.term[t].coef, sum[c], total[c]);
        }
        if (a.mode == FWD_STORE) {
            st4(a.out + e, total);
        } else if (a.mode == FWD_ACCUM) {
            ld4(a.out + e, v);
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += total[c];
            st4(a.out + e, v);
        } else {
            float yo[4], bd[4], yn[4], ps[4];
            ld4(a.y_old + e, yo);
            ld4(a.bdat + e, bd);
            if (a.compact) {
                ld4(a.psi + e, ps);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float zeta = total[c] + ps[c];
                    yn[c] = (yo[c] + a.sigma * zeta - a.sigma * bd[c]) * a.inv1ps;
                    ps[c] = fmaf(a.p[a.kidx], total[c], ps[c]);
                }
                st4(a.psi + e, ps);
            } else {
                float avg[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int j = 0; j < a.r; ++j) {
                    ld4(a.psi + (size_t)j * m + e, v);
#pragma unroll
                    for (int c = 0; c < 4; ++c) avg[c] = fmaf(a.p[j], v[c], avg[c]);
                }
                ld4(a.psi + (size_t)a.kidx * m + e, ps);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    // outside the measurement block: zeta is the average alone
                    const bool in = (long long)(e + c) >= a.e0 && (long long)(e + c) < a.e1;
                    const float zeta = in ? (total[c] - ps[c]) + avg[c] : avg[c];
                    yn[c] = (yo[c] + a.sigma * zeta - a.sigma * bd[c]) * a.inv1ps;
                    if (in) ps[c] = total[c];
                }
                st4(a.psi + (size_t)a.kidx * m + e, ps);
            }
            st4(a.y_new + e, yn);
        }
    }
}

__global__ void __launch_bounds__(256) k_fwd_reduce4(FwdArgs a) { fwd_reduce4_body(a, this_block()); }

// ------------------------------------------------------ exact transpose

// Ray-driven transpose with exclusive ownership: every wavefront owns two
// level-l image rows (columns, for column-stepping angles) as LDS
// accumulators and scatters into them the two taps of every sample of its
// angle group.  Within one instruction the lanes' rays are `phases` bins
// apart, so their coordinates differ by at least a pixel and no two lanes
// touch the same pixel; each pixel therefore receives its contributions in
// program order and the result is deterministic.  The weights come from the
// same fixed-point coordinate as the forward: the pair is an exact transpose.
// Sinogram values are read from global memory, one trip ahead of their use.
//
// Taps are not range-tested per sample.  Every bin of a wavefront's range
// (the bins of its workgroup's rows, or of its own R rows) reaches [-1, nl]
// at one of the workgroup's rows, and the coordinate moves by at most one
// pixel per row (|slope| <= 1 on the stepping axis), so at any row of the
// workgroup the left tap lies in [-(rows+1), nl+rows-1].  Each LDS row of
// S = nl + 2 kBpPad cells puts kBpPad >= rows+3 spare cells on both
// sides; a tap's cell index (tap + kBpPad) is clamped as an unsigned number to
// S-2, so every tap outside the row (beyond either end) lands in the last two
// cells, which no in-range tap reaches and which are never read back.  Only
// lanes whose bin lies past the range (zero contributions) get there.
// Unclamped lanes stay on the bin lattice, so they never share a cell within
// one instruction.
// The tile shape (rows per wavefront R, wavefronts per workgroup W) is a
// template parameter; the launcher picks it per level.
#ifndef IMK_BP_CHUNKS
#define IMK_BP_CHUNKS 2
#endif
constexpr int kBpChunks = IMK_BP_CHUNKS;  // 64-ray chunks per trip of a wavefront
template <int R, int W>
struct BpShape {
    static constexpr int rows = R * W;   // rows of a workgroup
    static constexpr int pad = rows + 4;  // spare cells on each side of an LDS row
    static_assert(pad >= rows + 3, "sink cells must lie beyond every in-range tap");
};

// Bins whose coordinate at steps r0 .. r0+nr-1 can reach [-1, nl] (ray
// constants a, c and 1/b in FP32; margins of 0.01 pixel cover their rounding).
__device__ __forceinline__ void bin_range(float ka, float kcc, float kib, int r0, int nrows, int nl, int nd, int& blo,
                                          int& cnt)
{
    const float fnl = (float)nl, bmax = (float)(nd - 1);
    const float base0 = fmaf((float)r0, ka, kcc);
    const float base1 = base0 + (float)(nrows - 1) * ka;
    const float e0 = (-1.01f - base0) * kib, e1 = (fnl + 0.01f - base0) * kib;
    const float e2 = (-1.01f - base1) * kib, e3 = (fnl + 0.01f - base1) * kib;
    blo = (int)fminf(fmaxf(ceilf(fminf(fminf(e0, e1), fminf(e2, e3))), 0.0f), bmax + 1.0f);
    const int bhi = (int)fmaxf(fminf(floorf(fmaxf(fmaxf(e0, e1), fmaxf(e2, e3))), bmax), -1.0f);
    cnt = bhi - blo + 1;
}



// One trip of a wavefront over CH chunks of 64 rays and its R rows (chains
// chunk-major): both taps of every sample, as two
// read-modify-write phases.  U[c] is chain c's shifted coordinate, wy[h] the
// weighted sinogram value of chunk h's ray (zero past the bin range).  With
// CLAMP the cell index is clamped (lanes past the range); without it every
// lane of the trip is in range and its taps lie inside the padded row.
template <int R, int CH, bool CLAMP>
__device__ __forceinline__ void scatter_trip(float* rows, int S, const long long* U, const float* wy)
{
    constexpr int NC = CH * R;
    int cl[NC];
    float omw[NC], cw[NC], wys[CH];
#pragma unroll
    for (int h = 0; h < CH; ++h) wys[h] = wy[h] * kTwoM32;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const unsigned hi = (unsigned)(U[c] >> 32);
        // unsigned clamp: taps past either end land in the last two cells
        const unsigned jj = CLAMP ? min(hi, (unsigned)(S - 2)) : hi;
        const float cu = (float)(unsigned)(U[c] & 0xffffffffLL);
        cl[c] = (c % R) * S + (int)jj;  // chains run over chunks, then rows
        cw[c] = cu;
        omw[c] = fmaf(cu, -kTwoM32, 1.0f);  // 1 - w, exactly as in the forward
    }
    float old[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) old[c] = rows[cl[c]];
#pragma unroll
    for (int c = 0; c < NC; ++c) rows[cl[c]] = fmaf(omw[c], wy[c / R], old[c]);
    IMK_LDS_ORDER();
#pragma unroll
    for (int c = 0; c < NC; ++c) old[c] = rows[cl[c] + 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) rows[cl[c] + 1] = fmaf(cw[c], wys[c / R], old[c]);
    IMK_LDS_ORDER();
}

__device__ __forceinline__ long long uniform64(long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffLL));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Raw buffer view of n floats: loads at or past the end return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t float_buffer(const float* base, int n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, n * 4, 0x00020000);
}

// The whole byte offset goes in the per-lane operand, which is the part the
// range check covers.
__device__ __forceinline__ float buffer_float(__amdgpu_buffer_rsrc_t r, int byte_offset)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_offset, 0, 0));
}

#ifndef IMK_BP_RUNS_MIN_P
#define IMK_BP_RUNS_MIN_P 3
#endif
// Angles whose rays are at least this many bins per pixel apart take runs.
constexpr int kBpRunsMinP = IMK_BP_RUNS_MIN_P;

// Run form of the scatter, for angles with `phases` P >= kBpRunsMinP (coarse
// levels, where neighbouring rays are less than a pixel apart).  Lane k
// takes the P consecutive bins that start P k bins into the trip: together
// they span less than one pixel ((P-1)|B| < 1 exactly, in the fixed-point
// coordinate), so on each row their taps fall in three cells base..base+2.
// The lane sums its contributions to those cells in registers and adds them
// to LDS in three read-modify-write phases; bases of different lanes are at
// least a pixel apart, so no two lanes share a cell in a phase.  A run costs
// three LDS updates per row instead of 2P.  Lanes past the bin range read
// zero sinogram values and have their base clamped (as an unsigned number)
// to S-3, the last three cells of the row.  One chunk of 64 runs per trip
// keeps the lanes busy when a range holds few runs.
template <int R>
__device__ __forceinline__ void scatter_runs(float* rows, int S, long long urow, long long afx, long long bfx,
                                             int blo, int cnt, int P, float kw, __amdgpu_buffer_rsrc_t yr,
                                             int lane)
{
    const int shift = bfx < 0 ? 1 : 0;  // a falling coordinate: the window starts one cell lower
    for (int c0 = 0; c0 < cnt; c0 += 64 * P) {
        long long U[R];
        unsigned base[R];
        int cl[R];
        // per row: the run's left-tap and right-tap totals, and the parts of
        // them from samples past the crossing into the next cell (the run
        // crosses at most once); then base gets tl - al, base+1 gets
        // (tr - ar) + al and base+2 gets ar.  A run of one sample gives its
        // two weights exactly, so every matrix entry is the forward's.
        float tl[R], tr[R], al[R], ar[R];
        const long long u0 = urow + (long long)(blo + c0 + lane * P) * bfx;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            U[rr] = u0 + rr * afx;
            base[rr] = (unsigned)(U[rr] >> 32) - (unsigned)shift;
            cl[rr] = rr * S + (int)min(base[rr], (unsigned)(S - 3));
            tl[rr] = tr[rr] = al[rr] = ar[rr] = 0.0f;
        }
        const int yb = (c0 + lane * P) * 4;
        float ynext = buffer_float(yr, yb);
        for (int t = 0; t < P; ++t) {
            const float wy = kw * ynext;
            const float wys = wy * kTwoM32;
            ynext = buffer_float(yr, yb + (t + 1) * 4);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const float cu = (float)(unsigned)(U[rr] & 0xffffffffLL);
                const float t0 = fmaf(cu, -kTwoM32, 1.0f) * wy;  // (1 - w) y, as in the forward
                const float t1 = cu * wys;                       // w y
                const float up = (unsigned)(U[rr] >> 32) != base[rr] ? 1.0f : 0.0f;  // taps at base+1, base+2
                tl[rr] += t0;
                tr[rr] += t1;
                al[rr] = fmaf(up, t0, al[rr]);
                ar[rr] = fmaf(up, t1, ar[rr]);
                U[rr] += bfx;
            }
        }
        float old[R];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) old[rr] = rows[cl[rr]];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) rows[cl[rr]] = old[rr] + (tl[rr] - al[rr]);
        IMK_LDS_ORDER();
#pragma unroll
        for (int rr = 0; rr < R; ++rr) old[rr] = rows[cl[rr] + 1];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) rows[cl[rr] + 1] = old[rr] + ((tr[rr] - ar[rr]) + al[rr]);
        IMK_LDS_ORDER();
#pragma unroll
        for (int rr = 0; rr < R; ++rr) old[rr] = rows[cl[rr] + 2];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) rows[cl[rr] + 2] = old[rr] + ar[rr];
        IMK_LDS_ORDER();
    }
}

// What a wavefront needs of one angle, tabulated in LDS by the workgroup:
// the bins of the workgroup's rows, or (wave_range) the FP32 constants from
// which each wavefront finds the bins of its own rows.
struct BpAngle {
    long long afx, bfx, cfx;  // fixed-point coordinate constants
    float w;                  // ray weight
    int phases;
    int ang;
    union {
        struct {
            int blo, cnt;
        } r;
        struct {
            float a, c, ib;
        } k;
    };
};
static_assert(sizeof(BpAngle) == 48, "BpAngle layout");
constexpr int kBpAngTab = 128;  // the most angles a workgroup tabulates at once

template <int R, int W>
__device__ __forceinline__ void bp_own_body(const BpOwnArgs& a, const Blk& bk, float* smem)
{
    constexpr int kBpRowsPerWave = R;
    constexpr int kBpRowsPerWg = BpShape<R, W>::rows;
    constexpr int kBpPad = BpShape<R, W>::pad;
    const int nl = a.n >> a.lvl;
    const int S = nl + 2 * kBpPad;
    float* acc = smem;                                     // kBpRowsPerWg x S
    BpAngle* tab = reinterpret_cast<BpAngle*>(smem + ((kBpRowsPerWg * S + 3) & ~3));
    const int bi = bk.x;    // band of kBpRowsPerWg rows
    const int gidx = bk.y;  // pass * G + angle group
    const int pass = gidx / a.G;
    const int g = gidx - pass * a.G;
    const int npass = pass == 0 ? a.split.nrow : a.split.ncol;
    // group g takes angles g, g + G, g + 2G, ... of its pass (the same mix
    // of steep and shallow angles in every group)
    const int nang = g < npass ? (npass - g + a.G - 1) / a.G : 0;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rwg = bi * kBpRowsPerWg;                 // first row of the workgroup
    const int nwg = min(kBpRowsPerWg, nl - rwg);
    const int r0 = rwg + wave * kBpRowsPerWave;        // first row of this wavefront
    const int nown = max(0, min(kBpRowsPerWave, nl - r0));
    float* rows = acc + (size_t)wave * kBpRowsPerWave * S;
    for (int q = lane; q < kBpRowsPerWave * S; q += 64) rows[q] = 0.0f;
    constexpr int NC = kBpChunks * kBpRowsPerWave;
    const int ntab = a.tab > 0 ? a.tab : kBpAngTab;
    for (int kb = 0; kb < nang; kb += ntab) {
        const int nk = min(ntab, nang - kb);
        __syncthreads();  // the previous block of the table is consumed
        for (int t = threadIdx.x; t < nk; t += blockDim.x) {
            const int ang = angle_of(a.split, pass, g + (kb + t) * a.G);
            const RayConst& kc = a.consts[(size_t)a.lvl * a.na + ang];
            BpAngle e;
            e.afx = kc.afx;
            e.bfx = kc.bfx;
            e.cfx = kc.cfx;
            e.w = kc.w;
            e.phases = kc.phases;
            e.ang = ang;
            if (a.wave_range) {
                e.k.a = kc.a;
                e.k.c = kc.c;
                e.k.ib = kc.ib;
            } else {
                bin_range(kc.a, kc.c, kc.ib, rwg, nwg, nl, a.nd, e.r.blo, e.r.cnt);
            }
            tab[t] = e;
        }
        __syncthreads();
        if (nown == 0) continue;
        for (int t = 0; t < nk; ++t) {
            const BpAngle& e = tab[t];
            int blo, cnt;
            if (a.wave_range) {
                // the bins that reach this wavefront's own rows: a tighter
                // range where the workgroup's rows are a large part of the
                // image (fewer idle lanes), at about 30 instructions per angle
                bin_range(__builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e.k.a))),
                          __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e.k.c))),
                          __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e.k.ib))),
                          r0, nown, nl, a.nd, blo, cnt);
            } else {
                blo = e.r.blo;
                cnt = e.r.cnt;
            }
            blo = __builtin_amdgcn_readfirstlane(blo);
            cnt = __builtin_amdgcn_readfirstlane(cnt);
            if (cnt <= 0) continue;
            const int ang = __builtin_amdgcn_readfirstlane(e.ang);
            const int P = __builtin_amdgcn_readfirstlane(e.phases);
            const float kw = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e.w)));
            // register copies: the ordering points below must not force reloads
            const long long afx = uniform64(e.afx), bfx = uniform64(e.bfx), cfx = uniform64(e.cfx);
            // sinogram values of the range, read straight from global memory
            // (L2/MALL-resident; lanes read consecutive bins), one trip ahead
            const __amdgpu_buffer_rsrc_t yr = float_buffer(a.y + (size_t)ang * a.nd + blo, cnt);
            const int vb = lane * P * 4;
            const long long urow = cfx + (long long)r0 * afx + ((long long)kBpPad << 32);
            if (kBpRunsMinP > 0 && P >= kBpRunsMinP) {
                scatter_runs<R>(rows, S, urow, afx, bfx, blo, cnt, P, kw, yr, lane);
                continue;
            }
            const long long cstep = (long long)64 * P * bfx;
            const int tstride = kBpChunks * 64 * P;
            const int full_end = cnt - (kBpChunks * 64 - 1) * P;  // trips starting below this are full
            for (int ph = 0; ph < P; ++ph) {
                // per chain (chunk h, row rr) the coordinate of its current ray,
                // shifted by kBpPad pixels so that its high word is the cell
                // index of the left tap within the padded LDS row
                long long U[NC];
                {
                    const long long u0 = urow + (long long)(blo + ph) * bfx + (long long)(lane * P) * bfx;
#pragma unroll
                    for (int h = 0; h < kBpChunks; ++h)
#pragma unroll
                        for (int rr = 0; rr < kBpRowsPerWave; ++rr) U[h * kBpRowsPerWave + rr] = u0 + h * cstep + rr * afx;
                }
                const long long trip = kBpChunks * cstep;
                float ynext[kBpChunks];
#pragma unroll
                for (int h = 0; h < kBpChunks; ++h) ynext[h] = buffer_float(yr, vb + (ph + h * 64 * P) * 4);
                int c0 = ph;
                for (; c0 < full_end; c0 += tstride) {
                    float wy[kBpChunks];
#pragma unroll
                    for (int h = 0; h < kBpChunks; ++h) {
                        wy[h] = kw * ynext[h];
                        ynext[h] = buffer_float(yr, vb + (c0 + tstride + h * 64 * P) * 4);
                    }
                    scatter_trip<R, kBpChunks, false>(rows, S, U, wy);
#pragma unroll
                    for (int c = 0; c < NC; ++c) U[c] += trip;
                }
                // the rest one chunk at a time, on the chains of chunk 0
                for (; c0 < cnt; c0 += 64 * P) {
                    float wy = kw * ynext[0];
                    ynext[0] = buffer_float(yr, vb + (c0 + 64 * P) * 4);
                    scatter_trip<R, 1, true>(rows, S, U, &wy);
#pragma unroll
                    for (int rr = 0; rr < kBpRowsPerWave; ++rr) U[rr] += cstep;
                }
            }
        }
    }
    // write back in image orientation: rows of the row pass directly, the
    // column pass through LDS as 8-column strips
    float* out = a.part + (size_t)gidx * nl * nl;
    if (pass == 0) {
        for (int rr = 0; rr < nown; ++rr)
            for (int q = lane; q < nl; q += 64) out[(size_t)(r0 + rr) * nl + q] = rows[rr * S + kBpPad + q];
    } else {
        __syncthreads();
        for (int q = threadIdx.x; q < nl * kBpRowsPerWg; q += blockDim.x) {
            const int i = q / kBpRowsPerWg, jj = q - i * kBpRowsPerWg;
            if (jj < nwg) out[(size_t)i * nl + rwg + jj] = acc[jj * S + kBpPad + i];
        }
    }
}

template <int R, int W>
__global__ void __launch_bounds__(64 * W) k_bp_own(BpOwnArgs a)
{
    extern __shared__ float smem[];
    bp_own_body<R, W>(a, this_block(), smem);
}

// A single-band forward's workgroups (its dual step in the epilogue), then
// the transpose's: on coarse levels both are small and latency-bound, and
// the step has one launch fewer.
template <int R, int W>
__global__ void __launch_bounds__(64 * W) k_bp_fwd(BpFwdArgs a)
{
    extern __shared__ float smem[];
    const int b = blockIdx.x;
    if (b < a.nfwd) {
        fwd_band_body(a.f, Blk{b % a.fgx, b / a.fgx, 0, a.fgx}, smem);
    } else {
        const int t = b - a.nfwd;
        bp_own_body<R, W>(a.b, Blk{t % a.bgx, t / a.bgx, 0, a.bgx}, smem);
    }
}

// The transpose's workgroups, then the forward's band reduce in the last
// ones: the memory-bound reduce fills the tail of the LDS-bound transpose,
// and the step has one launch fewer.
template <int R, int W>
__global__ void __launch_bounds__(64 * W) k_bp_red(BpRedArgs a)
{
    extern __shared__ float smem[];
    const int b = blockIdx.x;
    if (b < a.nbp) {
        bp_own_body<R, W>(a.b, Blk{b % a.bgx, b / a.bgx, 0, a.bgx}, smem);
    } else if (a.red4) {
        fwd_reduce4_body(a.f, Blk{b - a.nbp, 0, 0, a.nred});
    } else {
        fwd_reduce_body(a.f, Blk{b - a.nbp, 0, 0, a.nred});
    }
}

// c = sum over the nq partial images in a fixed order; coef * c is stored coarse
// (or into `tmp` for a later prolongation).  The nq partials are cut into S
// consecutive slices (S a power of two, chosen from the image size so that
// every level keeps about 2^18 threads busy): a workgroup of 1024 threads
// takes V 1024/S cells, each thread sums one slice of V cells in partial
// order, and the slice sums are added in slice order.
#ifndef IMK_BP_SUM_MAX_SLICES
#define IMK_BP_SUM_MAX_SLICES 64
#endif
constexpr int kBpSumMaxSlices = IMK_BP_SUM_MAX_SLICES;  // <= 1024, a power of two

// Slice sl of the nq partial images at the V consecutive cells from e,
// summed in partial order (V = 4: one 16-byte load per partial).
template <int V>
__device__ __forceinline__ void slice_sum(const BpOwnArgs& a, size_t d, size_t e, int q0, int q1, float* sum)
{
#pragma unroll
    for (int c = 0; c < V; ++c) sum[c] = 0.0f;
    if (e >= d) return;
    int q = q0;
    // eight partials loaded before any is added (their latencies overlap),
    // then added in partial order
    constexpr int U = 8;
    for (; q + U <= q1; q += U) {
        float v[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float* pp = a.part + (q + u) * d + e;
            if constexpr (V == 4)
                ld4(pp, v[u]);
            else
                v[u][0] = pp[0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < V; ++c) sum[c] += v[u][c];
    }
    for (; q < q1; ++q) {
        const float* pp = a.part + q * d + e;
        if constexpr (V == 4) {
            float v[4];
            ld4(pp, v);
#pragma unroll
            for (int c = 0; c < 4; ++c) sum[c] += v[c];
        } else {
            sum[0] += pp[0];
        }
    }
}

// Each thread sums its slice for V consecutive cells (V = 4 needs d a
// multiple of 4); the slices are then added one cell per thread.
template <int V>
__device__ __forceinline__ void bp_sum_body(const BpOwnArgs& a, float* tmp, int S, const Blk& bk)
{
    __shared__ float red[1024 * V];
    const int nl = a.n >> a.lvl;
    const size_t d = (size_t)nl * nl;
    const int per = 1024 / S;  // threads per slice
    const int sl = threadIdx.x / per;
    const int pi = threadIdx.x - sl * per;
    const size_t e = ((size_t)bk.x * per + pi) * V;
    float sum[V];
    slice_sum<V>(a, d, e, sl * a.nq / S, (sl + 1) * a.nq / S, sum);
#pragma unroll
    for (int c = 0; c < V; ++c) red[threadIdx.x * V + c] = sum[c];
    __syncthreads();
    // slice sums in slice order, one cell per thread
    const size_t e0 = (size_t)bk.x * per * V;
    const int ncell = (int)min((size_t)per * V, d - min(d, e0));
    for (int t = threadIdx.x; t < ncell; t += blockDim.x) {
        float cc = red[t];
        for (int k = 1; k < S; ++k) cc += red[k * per * V + t];
        const float v = a.coef * cc;
        float* o = (a.prolong ? tmp : a.out) + e0 + t;
        *o = a.accumulate && !a.prolong ? *o + v : v;
    }
}

template <int V>
__global__ void __launch_bounds__(1024) k_bp_sum(BpOwnArgs a, float* tmp, int S)
{
    bp_sum_body<V>(a, tmp, S, this_block());
}

// The ordered partial sum fused with the primal step of Alg. 1, for steps
// whose sketch needs one backprojection (a coarse sketch k > 0, or a single
// level): workgroup w sums its V 1024/S cells c of the level-l raw
// backprojection exactly as k_bp_sum does, forms g = 4^{-l} c, reads the old
// phi_k of its cells into LDS and refreshes them with g, then updates every
// full-resolution pixel of its cells as k_primal does (xi = (g - phi_k) +
// sum_j p_j phi_j with the old tables; x+ = (x - tau xi) * prox_scale, and
// xbar).  A cell's pixels and its phi_k entry belong to one workgroup, so
// the old table values it reads are never overwritten by another.
template <int V>
__device__ __forceinline__ void bp_sum_primal_body(const BpOwnArgs& a, int S, const PrimalArgs& p, const Blk& bk)
{
    __shared__ float red[1024 * V];
    __shared__ float gsh[1024 * V], own[1024 * V];
    const int l = a.lvl;
    const int nl = a.n >> l;
    const size_t d = (size_t)nl * nl;
    const int per = 1024 / S;  // threads per slice
    const int sl = threadIdx.x / per;
    const int pi = threadIdx.x - sl * per;
    const size_t e0 = (size_t)bk.x * per * V;  // the workgroup's first cell
    const size_t e = e0 + (size_t)pi * V;
    float sum[V];
    slice_sum<V>(a, d, e, sl * a.nq / S, (sl + 1) * a.nq / S, sum);
#pragma unroll
    for (int c = 0; c < V; ++c) red[threadIdx.x * V + c] = sum[c];
    __syncthreads();
    const long long koff = p.jblk * p.blk_stride + p.phi_off[p.kidx];
    const int ncell = (int)min((size_t)per * V, d - min(d, e0));
    // slice sums in slice order, one cell per thread
    for (int t = threadIdx.x; t < ncell; t += blockDim.x) {
        float cc = red[t];
        for (int k = 1; k < S; ++k) cc += red[k * per * V + t];
        const float g = (a.coef * cc) * (1.0f / (float)(1 << (2 * l)));
        gsh[t] = g;
        own[t] = p.phi[koff + e0 + t];
        p.phi[koff + e0 + t] = g;  // phi_k refresh
    }
    __syncthreads();
    // the cells' pixels: 2^l rows of 2^l pixels per cell, cells in order
    const int L2 = 1 << l;
    for (int q = threadIdx.x; q < ncell * L2 * L2; q += blockDim.x) {
        const int fr = q / (ncell * L2), rem = q - fr * (ncell * L2);
        const int c = rem >> l, fc = rem - (c << l);
        const size_t ec = e0 + c;
        const int ci = (int)(ec / nl), cj = (int)(ec - (size_t)ci * nl);
        const int i = ci * L2 + fr, j = cj * L2 + fc;
        const size_t pix = (size_t)i * p.n + j;
        const float g = gsh[c];
        float avg = 0.0f, ownv = 0.0f;
        if (p.nblk == 1) {
            // every level's entry loaded before the first is used (level k's,
            // already refreshed, is replaced by its old value kept in LDS),
            // then combined in level order
            ownv = own[c];
            float ph[IMASK_MAX_LEVELS];
#pragma unroll
            for (int cc = 0; cc < IMASK_MAX_LEVELS; ++cc) {
                if (cc >= p.r) break;
                const int lc = p.lvl[cc];
                const size_t cell = cc == 0 ? pix : (size_t)(i >> lc) * (p.n >> lc) + (j >> lc);
                ph[cc] = p.phi[p.phi_off[cc] + cell];
            }
#pragma unroll
            for (int cc = 0; cc < IMASK_MAX_LEVELS; ++cc) {
                if (cc >= p.r) break;
                avg = fmaf(p.pavg[cc], cc == p.kidx ? ownv : ph[cc], avg);
            }
        } else {
            for (int cc = 0; cc < p.r; ++cc) {
                const int lc = p.lvl[cc];
                const size_t cell = cc == 0 ? pix : (size_t)(i >> lc) * (p.n >> lc) + (j >> lc);
                for (int bb = 0; bb < p.nblk; ++bb) {  // one table per measurement block
                    float ph;
                    if (cc == p.kidx && bb == p.jblk) {
                        ph = own[c];
                        ownv = ph;
                    } else {
                        ph = p.phi[bb * p.blk_stride + p.phi_off[cc] + cell];
                    }
                    avg = fmaf(p.pavg[cc], ph, avg);
                }
            }
        }
        const float xi = (g - ownv) + avg;
        const float xo = p.x_old[pix];
        const float xn = (xo - p.tau * xi) * p.prox_scale;
        p.x_out[pix] = xn;
        if (p.xbar) p.xbar[pix] = xn + p.theta * (xn - xo);
    }
}

template <int V>
__global__ void __launch_bounds__(1024) k_bp_sum_primal(BpOwnArgs a, int S, PrimalArgs p)
{
    bp_sum_primal_body<V>(a, S, p, this_block());
}

__global__ void k_prolong_acc(const float* in, float* out, int n, int lvl, int accumulate)
{
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)n * n) return;
    const int i = (int)(q / n), j = (int)(q % n);
    const float v = in[(size_t)(i >> lvl) * (n >> lvl) + (j >> lvl)];
    out[q] = accumulate ? out[q] + v : v;
}

// ------------------------------------------------------------ primal step

// Forms phi_new = K_k^T y at full resolution from the raw backprojections,
// the SAGA estimate xi with the old tables, v = x - tau xi, and writes
// prox_scale * v; then refreshes table k.  One workgroup per T x T tile
// (T a multiple of every level's block, so coarse cells never straddle).
__device__ __forceinline__ void primal_tile(const PrimalArgs& a, int ty, int tx, const float* pyr);

__device__ __forceinline__ void primal_body(const PrimalArgs& a, const Blk& bk, float* pyr)
{
    const int tiles = a.n / a.T;
    const int ty = bk.x / tiles, tx = bk.x - ty * tiles;
    const bool paper_full = (a.kidx == 0 && a.full_mode == IMASK_FULL_PAPER && a.r > 1);
    if (paper_full) {
        load_tile(pyr, a.craw[0], a.n, a.T, ty, tx);
        build_pyramid(pyr, a.T, a.pyr_levels);
    }
    primal_tile(a, ty, tx, pyr);
}

// The primal step of one T x T tile (tile row ty, column tx); for a PAPER
// full-resolution sketch `pyr` holds the tile's raw backprojection and its
// 2x2-mean pyramid.
__device__ __forceinline__ void primal_tile(const PrimalArgs& a, int ty, int tx, const float* pyr)
{
    const bool paper_full = (a.kidx == 0 && a.full_mode == IMASK_FULL_PAPER && a.r > 1);
    const float ip0 = 1.0f / a.p[0];
    for (int qq = threadIdx.x; qq < a.T * a.T; qq += blockDim.x) {
        const int ti = qq / a.T, tj = qq - ti * a.T;
        const int i = ty * a.T + ti, j = tx * a.T + tj;
        const size_t pix = (size_t)i * a.n + j;
        float g;
        if (a.kidx > 0) {
            const int l = a.lvl[a.kidx];
            const int nl = a.n >> l;
            g = a.craw[a.kidx][(size_t)(i >> l) * nl + (j >> l)] * (1.0f / (float)(1 << (2 * l)));
        } else if (a.r == 1) {
            g = a.craw[0][pix];
        } else if (paper_full) {
            float acc = pyr[qq];
            for (int c = 1; c < a.r; ++c) {
                const int l = a.lvl[c];
                const int tc = a.T >> l;
                acc -= a.p[c] * pyr[pyr_offset(a.T, l) + (ti >> l) * tc + (tj >> l)];
            }
            g = acc * ip0;
        } else {
            float acc = a.craw[0][pix];
            for (int c = 1; c < a.r; ++c) {
                const int l = a.lvl[c];
                const int nl = a.n >> l;
                acc -= a.p[c] * (1.0f / (float)(1 << (2 * l))) * a.craw[c][(size_t)(i >> l) * nl + (j >> l)];
            }
            g = acc * ip0;
        }
        float avg = 0.0f, own = 0.0f;
        if (a.nblk == 1) {
            // every level's entry loaded before the first is used, then
            // combined in level order
            float ph[IMASK_MAX_LEVELS];
#pragma unroll
            for (int c = 0; c < IMASK_MAX_LEVELS; ++c) {
                if (c >= a.r) break;
                const int l = a.lvl[c];
                const size_t cell = c == 0 ? pix : (size_t)(i >> l) * (a.n >> l) + (j >> l);
                ph[c] = a.phi[a.phi_off[c] + cell];
            }
#pragma unroll
            for (int c = 0; c < IMASK_MAX_LEVELS; ++c) {
                if (c >= a.r) break;
                avg = fmaf(a.pavg[c], ph[c], avg);
                if (c == a.kidx) own = ph[c];
            }
        } else {
            for (int c = 0; c < a.r; ++c) {
                const int l = a.lvl[c];
                const size_t cell = c == 0 ? pix : (size_t)(i >> l) * (a.n >> l) + (j >> l);
                for (int b = 0; b < a.nblk; ++b) {  // one table per measurement block
                    const float ph = a.phi[b * a.blk_stride + a.phi_off[c] + cell];
                    avg = fmaf(a.pavg[c], ph, avg);
                    if (c == a.kidx && b == a.jblk) own = ph;
                }
            }
        }
        const float xi = (g - own) + avg;
        const float xo = a.x_old[pix];
        const float xn = (xo - a.tau * xi) * a.prox_scale;
        a.x_out[pix] = xn;
        if (a.xbar) a.xbar[pix] = xn + a.theta * (xn - xo);
        if (a.kidx == 0) a.phi[a.jblk * a.blk_stride + a.phi_off[0] + pix] = g;
    }
    if (a.kidx > 0) {
        __syncthreads();  // every old phi_k value of this tile has been read
        const int l = a.lvl[a.kidx];
        const int nl = a.n >> l, tl = a.T >> l;
        const float s = 1.0f / (float)(1 << (2 * l));
        for (int qq = threadIdx.x; qq < tl * tl; qq += blockDim.x) {
            const int ci = ty * tl + qq / tl, cj = tx * tl + (qq % tl);
            const size_t c = (size_t)ci * nl + cj;
            a.phi[a.jblk * a.blk_stride + a.phi_off[a.kidx] + c] = a.craw[a.kidx][c] * s;
        }
    }
}

__global__ void __launch_bounds__(256) k_primal(PrimalArgs a)
{
    extern __shared__ float pyr[];
    primal_body(a, this_block(), pyr);
}

// Level 0 of a PAPER full-resolution sketch: the workgroup's 32 x 32 tile
// of the raw backprojection, each pixel's partial images summed in a fixed
// order (kSumTileSlices consecutive slices of the partials, each summed in
// partial order, then the slices in order; 16-byte loads, rows of the tile
// are whole 128-byte lines), scaled by the transpose's coefficient, into
// the tile pyramid; then the primal step of the tile as k_primal takes it.
// The raw backprojection itself is never stored.
constexpr int kSumTileSlices = 4;
constexpr int kSumTileThreads = 1024;
__device__ __forceinline__ void sum_primal_tile_body(const BpOwnArgs& a, const PrimalArgs& p, const Blk& bk,
                                                     float* pyr)
{
    constexpr int T = 32;  // plan_sum_primal_tile
    const int tiles = p.n / T;
    const int ty = bk.x / tiles, tx = bk.x - ty * tiles;
    const size_t d = (size_t)p.n * p.n;
    float* red = pyr + 2 * T * T;  // kSumTileSlices x T^2 slice sums (the pyramid needs under 2 T^2)
    {
        const int per = T * T / 4;  // threads of one slice: four pixels each
        const int sl = threadIdx.x / per, f = threadIdx.x - sl * per;
        const int qq = 4 * f;
        const int ti = qq / T, tj = qq - ti * T;
        const float* pp = a.part + (size_t)(ty * T + ti) * p.n + tx * T + tj;
        const int q0 = sl * a.nq / kSumTileSlices, q1 = (sl + 1) * a.nq / kSumTileSlices;
        float sum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        int q = q0;
        for (; q + 8 <= q1; q += 8) {  // eight loads in flight, added in partial order
            float v[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u) ld4(pp + (size_t)(q + u) * d, v[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < 4; ++c) sum[c] += v[u][c];
        }
        for (; q < q1; ++q) {
            float v[4];
            ld4(pp + (size_t)q * d, v);
#pragma unroll
            for (int c = 0; c < 4; ++c) sum[c] += v[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) red[sl * T * T + qq + c] = sum[c];
    }
    __syncthreads();
    for (int qq = threadIdx.x; qq < T * T; qq += blockDim.x) {
        float c = red[qq];
        for (int k = 1; k < kSumTileSlices; ++k) c += red[k * T * T + qq];
        pyr[qq] = a.coef * c;
    }
    build_pyramid(pyr, T, p.pyr_levels);
    primal_tile(p, ty, tx, pyr);
}

__global__ void __launch_bounds__(kSumTileThreads) k_sum_primal_tile(SumTileArgs a)
{
    extern __shared__ float pyr[];
    sum_primal_tile_body(a.a, a.p, this_block(), pyr);
}

// ------------------------------------- several levels of one sketch per launch

// The part a block belongs to, and its block within that part's own grid.
__device__ __forceinline__ Blk multi_block(const int* start, const int* gx, int n, int& t)
{
    const int b = blockIdx.x;
    t = 0;
    while (t + 1 < n && b >= start[t + 1]) ++t;
    const int local = b - start[t];
    return Blk{local % gx[t], local / gx[t], 0, gx[t]};
}

__global__ void __launch_bounds__(1024) k_fwd_band_multi(FwdMultiArgs m)
{
    extern __shared__ float band[];
    int t;
    const Blk bk = multi_block(m.start, m.gx, m.n, t);
    fwd_band_body(m.t[t], bk, band);
}

template <int R, int W>
__global__ void __launch_bounds__(64 * W) k_bp_own_multi(BpMultiArgs m)
{
    extern __shared__ float smem[];
    int t;
    const Blk bk = multi_block(m.start, m.gx, m.n, t);
    bp_own_body<R, W>(m.t[t], bk, smem);
}

__global__ void __launch_bounds__(1024) k_bp_sum_multi(SumMultiArgs m)
{
    int t = 0;
    const int b = blockIdx.x;
    while (t + 1 < m.n && b >= m.start[t + 1]) ++t;
    const int local = b - m.start[t];
    const Blk bk{local, 0, 0, m.start[t + 1] - m.start[t]};
    if (m.v[t] == 4)
        bp_sum_body<4>(m.t[t].a, m.t[t].tmp, m.t[t].S, bk);
    else
        bp_sum_body<1>(m.t[t].a, m.t[t].tmp, m.t[t].S, bk);
}

// ------------------------------------------------------------ smoothed TV

// J FISTA iterations of the prox of tau*(w TV_eps + lam/2 |.|^2) on one
// 32 x 32 output tile; the workgroup holds the tile plus a J-pixel halo in
// LDS, so the whole inner solve reads v and u0 once and writes the result
// once.  Every thread keeps a fixed set of cells (their input v, previous
// iterate and neighbour masks in registers) and updates them at every
// iteration: a cell at the tile's edge sees no neighbour beyond it, an error
// that moves inward one pixel per iteration and so never reaches the output
// tile, which lies J pixels inside.
#ifndef IMK_TV_TILE
#define IMK_TV_TILE 32
#endif
#ifndef IMK_TV_THREADS
#define IMK_TV_THREADS 1024
#endif
constexpr int kTvTile = IMK_TV_TILE;
constexpr int kTvThreads = IMK_TV_THREADS;
// cells per thread: the tile with the largest halo either kernel uses (J + 1)
constexpr int kTvSideMax = kTvTile + 2 * (IMASK_MAX_TV_INNER + 1);
constexpr int kTvCells = (kTvSideMax * kTvSideMax + kTvThreads - 1) / kTvThreads;

__global__ void __launch_bounds__(kTvThreads) k_tv(TvArgs a)
{
    extern __shared__ float sm[];
    const int H = a.J;
    const int R = kTvTile + 2 * H;
    float* ys = sm;          // extrapolated point y of FISTA
    float* q1 = ys + R * R;  // normalised gradient, row direction
    float* q2 = q1 + R * R;  // normalised gradient, column direction
    const int tiles = (a.n + kTvTile - 1) / kTvTile;
    const int ty = blockIdx.x / tiles, tx = blockIdx.x - ty * tiles;
    const int gi0 = ty * kTvTile - H, gj0 = tx * kTvTile - H;
    const int n = a.n;
    const float eps2 = a.eps * a.eps;
    enum { kIn = 1, kDown = 2, kRight = 4, kUp = 8, kLeft = 16, kOut = 32 };
    int cell[kTvCells], flag[kTvCells], ring[kTvCells];
    // per cell in registers: input v, previous iterate, current y and its
    // normalised gradient (the LDS copies serve the neighbours)
    float vv[kTvCells], up[kTvCells], yk[kTvCells], g1[kTvCells], g2[kTvCells];
#pragma unroll
    for (int k = 0; k < kTvCells; ++k) {
        const int q = threadIdx.x + k * kTvThreads;
        flag[k] = 0;
        cell[k] = q;
        ring[k] = 0;
        vv[k] = up[k] = yk[k] = g1[k] = g2[k] = 0.0f;
        if (q >= R * R) continue;
        const int li = q / R, lj = q - li * R;
        ring[k] = min(min(li, lj), min(R - 1 - li, R - 1 - lj));
        const int gi = gi0 + li, gj = gj0 + lj;
        if (gi < 0 || gi >= n || gj < 0 || gj >= n) {
            ys[q] = 0.0f;
            continue;
        }
        flag[k] = kIn | (gi < n - 1 && li < R - 1 ? kDown : 0) | (gj < n - 1 && lj < R - 1 ? kRight : 0) |
                  (gi >= 1 && li >= 1 ? kUp : 0) | (gj >= 1 && lj >= 1 ? kLeft : 0) |
                  (li >= H && li < H + kTvTile && lj >= H && lj < H + kTvTile ? kOut : 0);
        vv[k] = a.v[(size_t)gi * n + gj];
        up[k] = a.u0[(size_t)gi * n + gj];
        yk[k] = up[k];
        ys[q] = up[k];
    }
    __syncthreads();
    // A cell's update reads cells at most one pixel away, so after iteration
    // t+1 only cells at least t+1 pixels inside the tile's edge (ring t+1)
    // still agree with the untiled iteration, and the output (ring J) needs
    // no others: iteration t updates rings > t, from gradients on rings >= t.
    for (int t = 0; t < a.J; ++t) {
        // q = grad y / sqrt(|grad y|^2 + eps^2), zero difference past the image
#pragma unroll
        for (int k = 0; k < kTvCells; ++k) {
            if (!(flag[k] & kIn) || ring[k] < t) continue;
            const int c = cell[k];
            const float yc = yk[k];
            const float d1 = (flag[k] & kDown) ? ys[c + R] - yc : 0.0f;
            const float d2 = (flag[k] & kRight) ? ys[c + 1] - yc : 0.0f;
            const float inv = rsqrtf(fmaf(d1, d1, fmaf(d2, d2, eps2)));
            g1[k] = d1 * inv;
            g2[k] = d2 * inv;
            q1[c] = g1[k];
            q2[c] = g2[k];
        }
        __syncthreads();
        const float beta = a.beta[t];
#pragma unroll
        for (int k = 0; k < kTvCells; ++k) {
            if (!(flag[k] & kIn) || ring[k] <= t) continue;
            const int c = cell[k];
            float div = -g1[k] - g2[k];  // grad^T q
            if (flag[k] & kUp) div += q1[c - R];
            if (flag[k] & kLeft) div += q2[c - 1];
            const float yc = yk[k];
            const float gh = (yc - vv[k]) + a.tau_w * div + a.tau_lam * yc;
            const float un = yc - a.invL * gh;
            yk[k] = un + beta * (un - up[k]);
            ys[c] = yk[k];
            up[k] = un;
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kTvCells; ++k) {
        if (!(flag[k] & kOut)) continue;
        const int li = cell[k] / R, lj = cell[k] - (cell[k] / R) * R;
        const size_t g = (size_t)(gi0 + li) * n + gj0 + lj;
        a.out[g] = up[k];
        if (a.xbar) a.xbar[g] = up[k] + a.theta * (up[k] - a.u0[g]);
    }
    if (a.prep_next) {
        // the next step's restriction of this output tile (tv_prep_fusable
        // holds: whole tiles, every output level inside one): the tile into
        // LDS, its 2x2-mean pyramid, and the same stores as k_prep
        float* pyr = sm;
#pragma unroll
        for (int k = 0; k < kTvCells; ++k) {
            if (!(flag[k] & kOut)) continue;
            const int li = cell[k] / R, lj = cell[k] - (cell[k] / R) * R;
            pyr[(li - H) * kTvTile + (lj - H)] = up[k];
        }
        build_pyramid(pyr, kTvTile, a.next.pyr_levels);
        prep_store(a.next, pyr, kTvTile, ty, tx);
    }
}


// Prox of gamma TV + chi_{>=0} at bt = v / scale (the paper's TV prior,
// Sec. 4.5), by J iterations of the fast gradient projection on the dual
// pair (p1, p2) (Beck-Teboulle), warm-started at the pair of the previous
// outer step.  Per iteration: u = max(0, bt - gamma grad^T r); the dual takes
// a step 1/(8 gamma) along grad u, is projected onto the unit disc per pixel
// and extrapolated.  Tiled like k_tv with a (J+1)-pixel halo: u reads r one
// pixel up/left, the dual step reads u one pixel down/right, so an edge
// error moves inward one pixel per iteration and the final u one more.
__global__ void __launch_bounds__(kTvThreads) k_tvd(TvdArgs a)
{
    extern __shared__ float sm[];
    const int H = a.J + 1;
    const int R = kTvTile + 2 * H;
    float* r1 = sm;          // extrapolated dual, row differences
    float* r2 = r1 + R * R;  // extrapolated dual, column differences
    float* uu = r2 + R * R;  // primal u(r)
    const int tiles = (a.n + kTvTile - 1) / kTvTile;
    const int ty = blockIdx.x / tiles, tx = blockIdx.x - ty * tiles;
    const int gi0 = ty * kTvTile - H, gj0 = tx * kTvTile - H;
    const int n = a.n;
    const size_t d = (size_t)n * n;
    enum { kIn = 1, kDown = 2, kRight = 4, kUp = 8, kLeft = 16, kOut = 32 };
    int cell[kTvCells], flag[kTvCells];
    // per cell in registers: prox input, dual iterate, extrapolated dual and
    // u (the LDS copies serve the neighbours)
    float bt[kTvCells], p1[kTvCells], p2[kTvCells], e1[kTvCells], e2[kTvCells], uk[kTvCells];
#pragma unroll
    for (int k = 0; k < kTvCells; ++k) {
        const int q = threadIdx.x + k * kTvThreads;
        flag[k] = 0;
        cell[k] = q;
        bt[k] = p1[k] = p2[k] = e1[k] = e2[k] = uk[k] = 0.0f;
        if (q >= R * R) continue;
        const int li = q / R, lj = q - li * R;
        const int gi = gi0 + li, gj = gj0 + lj;
        if (gi < 0 || gi >= n || gj < 0 || gj >= n) {
            r1[q] = r2[q] = uu[q] = 0.0f;
            continue;
        }
        const bool down = gi < n - 1, right = gj < n - 1;  // differences that exist in the image
        flag[k] = kIn | (down && li < R - 1 ? kDown : 0) | (right && lj < R - 1 ? kRight : 0) |
                  (gi >= 1 && li >= 1 ? kUp : 0) | (gj >= 1 && lj >= 1 ? kLeft : 0) |
                  (li >= H && li < H + kTvTile && lj >= H && lj < H + kTvTile ? kOut : 0);
        const size_t g = (size_t)gi * n + gj;
        bt[k] = a.v[g] * a.inv_scale;
        p1[k] = down ? a.pin[g] : 0.0f;
        p2[k] = right ? a.pin[d + g] : 0.0f;
        e1[k] = p1[k];
        e2[k] = p2[k];
        r1[q] = p1[k];
        r2[q] = p2[k];
    }
    __syncthreads();
    for (int t = 0; t < a.J; ++t) {
        // u = max(0, bt - gamma grad^T r)
#pragma unroll
        for (int k = 0; k < kTvCells; ++k) {
            if (!(flag[k] & kIn)) continue;
            const int c = cell[k];
            float gt = -e1[k] - e2[k];
            if (flag[k] & kUp) gt += r1[c - R];
            if (flag[k] & kLeft) gt += r2[c - 1];
            uk[k] = fmaxf(0.0f, bt[k] - a.gamma * gt);
            uu[c] = uk[k];
        }
        __syncthreads();
        const float beta = a.beta[t];
#pragma unroll
        for (int k = 0; k < kTvCells; ++k) {
            if (!(flag[k] & kIn)) continue;
            const int c = cell[k];
            const float uc = uk[k];
            const float g1 = (flag[k] & kDown) ? uu[c + R] - uc : 0.0f;
            const float g2 = (flag[k] & kRight) ? uu[c + 1] - uc : 0.0f;
            const float a1 = fmaf(g1, a.inv8g, e1[k]);
            const float a2 = fmaf(g2, a.inv8g, e2[k]);
            const float sc = fminf(1.0f, rsqrtf(fmaf(a1, a1, a2 * a2)));  // 1 / max(1, |a|)
            const float n1 = a1 * sc, n2 = a2 * sc;
            e1[k] = n1 + beta * (n1 - p1[k]);
            e2[k] = n2 + beta * (n2 - p2[k]);
            r1[c] = e1[k];
            r2[c] = e2[k];
            p1[k] = n1;
            p2[k] = n2;
        }
        __syncthreads();
    }
    // u(p_J) on the output tile, and the dual pair for the next outer step
#pragma unroll
    for (int k = 0; k < kTvCells; ++k) {
        if (!(flag[k] & kIn)) continue;
        r1[cell[k]] = p1[k];
        r2[cell[k]] = p2[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTvCells; ++k) {
        if (!(flag[k] & kOut)) continue;
        const int c = cell[k];
        float gt = -r1[c] - r2[c];
        if (flag[k] & kUp) gt += r1[c - R];
        if (flag[k] & kLeft) gt += r2[c - 1];
        const float u = fmaxf(0.0f, bt[k] - a.gamma * gt);
        const int li = c / R, lj = c - li * R;
        const size_t g = (size_t)(gi0 + li) * n + gj0 + lj;
        a.out[g] = u;
        if (a.xbar) a.xbar[g] = u + a.theta * (u - a.u0[g]);
        a.pout[g] = p1[k];
        a.pout[d + g] = p2[k];
    }
}

// ------------------------------------------------------------- resampling

__global__ void k_prolong(const float* in, float* out, int n, int lvl, float coef)
{
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)n * n) return;
    const int i = (int)(q / n), j = (int)(q % n);
    const int nl = n >> lvl;
    out[q] = coef * in[(size_t)(i >> lvl) * nl + (j >> lvl)];
}

__global__ void k_project_block(const float* in, float* out, int n, int lvl)
{
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)n * n) return;
    const int i = (int)(q / n), j = (int)(q % n);
    const int f = 1 << lvl;
    const int i0 = (i >> lvl) << lvl, j0 = (j >> lvl) << lvl;
    float s = 0.0f;
    for (int di = 0; di < f; ++di)
        for (int dj = 0; dj < f; ++dj) s += in[(size_t)(i0 + di) * n + j0 + dj];
    out[q] = s / (float)(f * f);
}

// ------------------------------------------------------- vector utilities

// y += a x
__global__ void k_axpy(float* y, const float* x, float a, size_t n)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        y[q] = fmaf(a, x[q], y[q]);
}

// x *= a
__global__ void k_scale(float* x, float a, size_t n)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        x[q] *= a;
}

// x[q] = uniform(-1, 1) from SplitMix64 of (seed, q)
__global__ void k_fill_random(float* x, size_t n, unsigned long long seed)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        unsigned long long z = seed + (q + 1) * 0x9E3779B97F4A7C15ULL;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        x[q] = (float)((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
    }
}

// Per-block FP64 partial sums of a[q] * b[q] (fixed block count, fixed order).
constexpr int kDotBlocks = 256;
__global__ void __launch_bounds__(256) k_dot_partial(const float* a, const float* b, size_t n, double* part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        acc += (double)a[q] * (double)b[q];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_dot_final(const double* part, double* out)
{
    __shared__ double red[kDotBlocks];
    red[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int w = kDotBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

bool tv_prep_fusable(int n, const PrepArgs& pa)
{
    if (n % kTvTile != 0 || pa.snap || (kTvTile >> pa.pyr_levels) < 1) return false;
    for (int o = 0; o < pa.nout; ++o)
        if ((kTvTile >> pa.out[o].lvl) < 1 || pa.out[o].lvl > pa.pyr_levels) return false;
    for (int c = 0; c < pa.ncomp; ++c)
        if (pa.comp_lvl[c] > pa.pyr_levels) return false;
    return true;
}
// the pyramid (a tile and its mean levels, under 4/3 of a tile) fits in the
// prox's LDS (three arrays of the tile with its halo)
static_assert(4 * kTvTile * kTvTile <= 3 * 3 * kTvTile * kTvTile, "pyramid fits the prox's LDS");

// ----------------------------------------------------------------- launchers

#ifndef IMK_TILE_MIN
#define IMK_TILE_MIN 16
#endif
int tile_side(int n, int lmax)
{
    int T = IMK_TILE_MIN;
    while (T > 16 && n % T != 0) T >>= 1;  // a divisor of n (n > 16 is a multiple of 16)
    if (T > n) T = n;
    while (T < (1 << lmax)) T <<= 1;
    return T;
}

hipError_t launch_consts(const imask_geometry& g, const Layout& L, float* work, hipStream_t s)
{
    const double side = 2.0 * (g.extent > 0 ? g.extent : 1.0);
    const double ds = g.det_spacing > 0 ? g.det_spacing : side / g.n;
    const int count = (L.lmax + 1) * g.n_angles;
    const AngleSplit sp = split_at(L, work);
    const double* th = L.listed ? (const double*)(work + L.angtab) : nullptr;
    hipLaunchKernelGGL(k_consts, dim3((count + 255) / 256), dim3(256), 0, s, g.n, g.n_angles, g.n_det, ds,
                       g.det_offset, side, th, sp.rows, L.lmax, (RayConst*)(work + L.consts));
    return hipGetLastError();
}

// flag = 1 if any of a[0..na) or b[0..nb) is a NaN or an infinity (all
// exponent bits set); flag is cleared beforehand by the caller.
__global__ void k_nonfinite(const float* a, size_t na, const float* b, size_t nb, int* flag)
{
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (size_t q = i0; q < na; q += stride) bad |= (__float_as_uint(a[q]) & 0x7f800000u) == 0x7f800000u;
    for (size_t q = i0; q < nb; q += stride) bad |= (__float_as_uint(b[q]) & 0x7f800000u) == 0x7f800000u;
    if (bad) flag[0] = 1;
}

hipError_t launch_nonfinite(const float* a, size_t na, const float* b, size_t nb, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, (float*)flag, (size_t)1, 0.0f);
    const size_t n = std::max(na, nb);
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_nonfinite, dim3(blocks), dim3(256), 0, s, a, na, b, nb, flag);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t count, float value, hipStream_t s)
{
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

static size_t pyramid_bytes(int T, int levels)
{
    size_t f = 0;
    for (int l = 0; l <= levels; ++l) f += (size_t)(T >> l) * (T >> l);
    return f * sizeof(float);
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t s)
{
    Launches r;
    plan_prep(a, r);
    return launch_records(r, s);
}

void plan_prep(const PrepArgs& a, Launches& out)
{
    Launch L;
    L.variant = V_PREP;
    const int tiles = a.n / a.T;
    L.gx = (unsigned)(tiles * tiles);
    L.block = 256;
    L.lds = (int)pyramid_bytes(a.T, a.pyr_levels);
    L.set(a);
    out.push_back(L);
}

// LDS budget of a forward band: up to 156 KB (one workgroup per CU, 7 bands
// of 74 rows) for 512-pixel rows, where fewer bands keep the partial
// sinograms few; 78 KB (two workgroups per CU, 4 bands) for 256-pixel rows;
// 64 KB for coarser levels, whose single large band would leave too few
// workgroups.
static int fwd_lds_bytes(int nl) { return (nl >= 512 ? 156 : nl >= 256 ? 78 : 64) * 1024; }

// The tuned shapes, per (level grid side, angles, bins); looked up on every
// launch, set rarely (imask_set_tiles).
struct TileEntry {
    int nl, na, nd;
    Tiles t;
};
static std::mutex g_tiles_mu;
static std::vector<TileEntry> g_tiles;

Tiles tiles_for(int nl, int na, int nd)
{
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    for (const TileEntry& e : g_tiles)
        if (e.nl == nl && e.na == na && e.nd == nd) return e.t;
    return Tiles{};
}

bool set_tiles(int nl, int na, int nd, const Tiles* t)
{
    if (t) {
        const int shape = t->bp_rows * 16 + t->bp_waves;
        const bool shape_ok = shape == 0 || shape == 2 * 16 + 8 || shape == 4 * 16 + 4 || shape == 2 * 16 + 4 ||
                              shape == 1 * 16 + 4;
        if (!shape_ok || t->bp_wg < 0 || t->bp_wg > 16384 || (t->bp_wg > 0 && t->bp_wg < 64) || t->fwd_lds_kb < 0 ||
            t->fwd_lds_kb > 156)
            return false;
    }
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    for (size_t q = 0; q < g_tiles.size(); ++q)
        if (g_tiles[q].nl == nl && g_tiles[q].na == na && g_tiles[q].nd == nd) {
            g_tiles.erase(g_tiles.begin() + q);
            break;
        }
    if (t && (t->bp_rows || t->bp_waves || t->bp_wg || t->fwd_lds_kb)) g_tiles.push_back(TileEntry{nl, na, nd, *t});
    return true;
}

// Levels of up to 1024 pixels per side take LDS bands (1024: 27 bands of
// 38 rows; measured 541 against 1688 us for the direct kernel at level 0 of
// 1024^2 / 1536 x 1536, 201 against 632 us for 768^2 / 1152 x 1152), as long
// as their partial sinograms stay within 512 MiB; longer rows take the
// direct kernel.
#ifndef IMK_BAND_MAX_SIDE
#define IMK_BAND_MAX_SIDE 1024
#endif
constexpr size_t kBandPartialBytes = (size_t)512 << 20;

static void bands_for_budget(int nl, size_t m, int bytes, int* bands, int* rows)
{
    const int maxr = bytes / (int)(sizeof(float) * (nl + kPad));
    const int nb = (nl + maxr - 1) / maxr;
    if (nl > IMK_BAND_MAX_SIDE || (nb > 1 && (size_t)nb * m * sizeof(float) > kBandPartialBytes)) {
        *bands = 1;  // the direct kernel: one partial
        *rows = 0;
        return;
    }
    *bands = nb;
    *rows = (nl + nb - 1) / nb;
}

void fwd_bands_default(int nl, int na, int nd, int* bands, int* rows)
{
    bands_for_budget(nl, (size_t)na * nd, fwd_lds_bytes(nl), bands, rows);
}

void fwd_bands(int nl, int na, int nd, int* bands, int* rows)
{
    const Tiles t = tiles_for(nl, na, nd);
    int bytes = fwd_lds_bytes(nl);
    if (t.fwd_lds_kb > 0) bytes = std::max(bytes, std::min(t.fwd_lds_kb, 156) * 1024);
    bands_for_budget(nl, (size_t)na * nd, bytes, bands, rows);
}

static hipError_t allow_lds(const void* fn, int bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// Arguments and launch shape of forward term t (band or direct kernel).
static Launch fwd_term_launch(const FwdArgs& a, int t, FwdBandArgs* args_out);
static void plan_reduce(const FwdArgs& a, Launches& out);

void plan_fwd_terms(const FwdArgs& a, Launches& out)
{
    for (int t = 0; t < a.nterms; ++t) out.push_back(fwd_term_launch(a, t, nullptr));
}

void plan_fwd_fused(const FwdArgs& a, Launches& out)
{
    FwdMultiArgs m{};
    Launch multi;
    multi.variant = V_FWD_MULTI;
    multi.block = 1024;
    for (int t = 0; t < a.nterms; ++t) {
        FwdBandArgs fb;
        const Launch L = fwd_term_launch(a, t, &fb);
        if (L.variant != V_FWD_BAND) {
            out.push_back(L);
            continue;
        }
        m.t[m.n] = fb;
        m.gx[m.n] = (int)L.gx;
        m.start[m.n + 1] = m.start[m.n] + (int)(L.gx * L.gy);
        multi.lds = std::max(multi.lds, L.lds);
        ++m.n;
    }
    if (m.n > 0) {
        multi.gx = (unsigned)m.start[m.n];
        multi.set(m);
        out.push_back(multi);
    }
    plan_reduce(a, out);
}

static Launch fwd_term_launch(const FwdArgs& a, int t, FwdBandArgs* args_out)
{
    const AngleSplit sp = a.split;
    {
        const FwdTerm& tm = a.term[t];
        FwdBandArgs fb{};
        fb.consts = a.consts;
        fb.fan = a.fan;
        fb.n = a.n;
        fb.na = a.na;
        fb.nd = a.nd;
        fb.lvl = tm.lvl;
        fb.img = tm.img;
        fb.imgT = tm.imgT;
        fb.part = tm.part;
        fb.split = sp;
        Launch L;
        if (tm.rows > 0) {
            const int nl = a.n >> tm.lvl;
            fb.R = tm.rows;
            fb.bands = tm.bands;
            // about 512 workgroups of 1024 threads over the angles this
            // launch projects (a measurement block covers only some of them);
            // 1024 where one band covers the level: its small band lets two
            // workgroups share a CU, and finer groups even out the CUs' work
            const int wg_target = tm.bands == 1 ? 1024 : 512;
            fb.apg = std::max(1, ((sp.nrow + sp.ncol) * tm.bands + wg_target - 1) / wg_target);
            fb.groups_row = (sp.nrow + fb.apg - 1) / fb.apg;
            fb.groups_col = (sp.ncol + fb.apg - 1) / fb.apg;
            L.variant = V_FWD_BAND;
            L.gx = (unsigned)tm.bands;
            L.gy = (unsigned)(fb.groups_row + fb.groups_col);
            L.block = 1024;
            L.lds = (int)(sizeof(float) * (size_t)fb.R * (nl + kPad));
        } else {
            const int wpa = (a.nd + 63) / 64;
            const long waves = (long)wpa * a.na;
            L.variant = V_FWD_DIRECT;
            L.gx = (unsigned)((waves + 3) / 4);
            L.block = 256;
            L.lds = 0;
        }
        L.set(fb);
        if (args_out) *args_out = fb;
        return L;
    }
}

// The band partials' ordered sum and the dual step (or store / accumulate).
static void plan_reduce(const FwdArgs& a, Launches& out)
{
    const size_t m = (size_t)a.na * a.nd;
    auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    const bool aligned = a.mode == FWD_DUAL ? al(a.y_old) && al(a.y_new) && al(a.bdat) && al(a.psi) : al(a.out);
    Launch L;
    if (m % 4 == 0 && aligned) {  // the workspace partials are 16-byte aligned too
        L.variant = V_RED4;
        L.gx = (unsigned)std::min<size_t>((m / 4 + 255) / 256, 8192);
    } else {
        L.variant = V_RED1;
        L.gx = (unsigned)std::min<size_t>((m + 255) / 256, 8192);
    }
    L.block = 256;
    L.set(a);
    out.push_back(L);
}

void plan_fwd(const FwdArgs& a, Launches& out)
{
    const size_t m = (size_t)a.na * a.nd;
    const bool single = a.mode == FWD_DUAL && a.nterms == 1 && a.term[0].rows > 0 && a.term[0].bands == 1 &&
                        !a.compact && !a.fan.ray && a.e0 == 0 && a.e1 == (long long)m && a.term[0].coef == 1.0f;
    if (single) {  // one band, one term: the dual step in the band kernel's epilogue, no reduce
        FwdBandArgs fb;
        Launch L = fwd_term_launch(a, 0, &fb);
        fb.dual = 1;
        fb.y_old = a.y_old;
        fb.bdat = a.bdat;
        fb.y_new = a.y_new;
        fb.psi = a.psi;
        fb.r = a.r;
        fb.kidx = a.kidx;
        for (int j = 0; j < IMASK_MAX_LEVELS; ++j) fb.p[j] = a.p[j];
        fb.sigma = a.sigma;
        fb.inv1ps = a.inv1ps;
        L.set(fb);
        out.push_back(L);
        return;
    }
    plan_fwd_terms(a, out);
    plan_reduce(a, out);
}

hipError_t launch_fwd_terms(const FwdArgs& a, hipStream_t s)
{
    if (a.fan.ray) {
        for (int t = 0; t < a.nterms; ++t) {
            const FwdTerm& tm = a.term[t];
            FwdBandArgs fb{};
            fb.consts = a.consts;
            fb.fan = a.fan;
            fb.n = a.n;
            fb.na = a.na;
            fb.nd = a.nd;
            fb.lvl = tm.lvl;
            fb.img = tm.img;
            fb.imgT = tm.imgT;
            fb.part = tm.part;
            fb.split = a.split;
            const size_t m = (size_t)(a.fan.vb - a.fan.va) * a.nd;
            if (tm.rows > 0) {
                // LDS bands of the level image, as the parallel beam's; about
                // 512 workgroups over bands, passes and view groups
                const int nl = a.n >> tm.lvl;
                const int nv = a.fan.vb - a.fan.va;
                fb.R = tm.rows;
                fb.bands = tm.bands;
                fb.groups_row = fb.groups_col = std::max(1, std::min(nv, 512 / (2 * tm.bands)));
                const int lds = (int)(sizeof(float) * (size_t)fb.R * (nl + kPad));
                hipError_t e = allow_lds((const void*)k_fwd_fan_band, lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(k_fwd_fan_band, dim3((unsigned)tm.bands, (unsigned)(2 * fb.groups_row)), dim3(1024),
                                   lds, s, fb);
            } else {
                hipLaunchKernelGGL(k_fwd_fan, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, fb);
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    Launches r;
    plan_fwd_terms(a, r);
    return launch_records(r, s);
}

hipError_t launch_fwd(const FwdArgs& a, hipStream_t s)
{
    Launches r;
    if (a.fan.ray) {  // fan-beam terms, then the same reduce
        const hipError_t e = launch_fwd_terms(a, s);
        if (e != hipSuccess) return e;
        plan_reduce(a, r);
    } else {
        plan_fwd(a, r);
    }
    return launch_records(r, s);
}

#ifndef IMK_BP_TARGET_WG
#define IMK_BP_TARGET_WG 1024
#endif
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per CU on gfx950

// Dynamic LDS of k_bp_own<R, W> for rows of nl pixels.
template <int R, int W>
static size_t scatter_lds(int nl, int tab = 0)
{
    using Sh = BpShape<R, W>;
    return sizeof(float) * ((size_t)Sh::rows * (nl + 2 * Sh::pad) + 3) + sizeof(BpAngle) * (tab > 0 ? tab : kBpAngTab);
}

// Ownership scatter with about IMK_BP_TARGET_WG workgroups: G angle groups
// per pass, 2 G N_l^2 partial images within the workspace's partial-image
// buffer.  A launch over part of the angles (a measurement block) keeps the
// same workgroup count: fewer angles per group, but fewer workgroups
// measured slower still.
template <int R, int W>
static void plan_scatter(BpOwnArgs& a, int nl, int lvl, int variant, int round, int target, Launches& out)
{
    using Sh = BpShape<R, W>;
    const int nb = (nl + Sh::rows - 1) / Sh::rows;
    const long long room = std::max<long long>(a.fan.part_floats, (long long)kPartImages * a.n * a.n) /
                           (2LL * nl * nl);
    const int gmax = (int)std::max(1LL, std::min<long long>({(long long)std::max(a.split.nrow, a.split.ncol), room,
                                                             1024LL}));
    a.G = std::max(1, std::min(gmax, (target + 2 * nb - 1) / (2 * nb)));
    a.nq = 2 * a.G;
    // per-wavefront bin ranges where a workgroup's rows are an eighth of the
    // image or more (512^2 / 720 x 768, level 3: 22.5 -> 19.0 us; level 0,
    // where the rows are 1/64 of it, pays 4% for the extra range work)
    a.wave_range = Sh::rows * 8 >= nl;
    // a table as long as the largest group: at level 0 of 512^2 / 720 x 768
    // (16 groups of at most 23 angles per pass) the workgroup's LDS falls
    // from 23 to 18 KB, so that eight workgroups share a CU instead of six
    a.tab = std::min(kBpAngTab, (std::max(a.split.nrow, a.split.ncol) + a.G - 1) / a.G);
    Launch L;
    L.variant = variant;
    L.round = round;
    L.gx = (unsigned)nb;
    L.gy = (unsigned)(2 * a.G);
    L.block = 64 * W;
    L.lds = (int)scatter_lds<R, W>(nl, a.tab);
    L.set(a);
    out.push_back(L);
}

static BpOwnArgs own_args(const BpArgs& ba)
{
    BpOwnArgs a{};
    a.consts = ba.consts;
    a.fan = ba.fan;
    a.n = ba.n;
    a.na = ba.na;
    a.nd = ba.nd;
    a.lvl = ba.lvl;
    a.y = ba.y;
    a.part = ba.part;
    a.split = ba.split;
    a.out = ba.out;
    a.coef = ba.coef;
    a.accumulate = ba.accumulate;
    a.prolong = ba.prolong;
    return a;
}

void plan_bp_main(const BpArgs& ba, int round, Launches& out, BpOwnArgs* used)
{
    BpOwnArgs a = own_args(ba);
    const int nl = ba.n >> ba.lvl;
    const Tiles t = tiles_for(nl, ba.na, ba.nd);
    const int target = t.bp_wg > 0 ? t.bp_wg : IMK_BP_TARGET_WG;
    // a tuned tile shape, where its rows fit in the 160 KB of LDS
    const int shape = t.bp_rows * 16 + t.bp_waves;
    if (shape == 2 * 16 + 8 && scatter_lds<2, 8>(nl) <= kLdsBytes) {
        plan_scatter<2, 8>(a, nl, ba.lvl, V_BP28, round, target, out);
    } else if (shape == 4 * 16 + 4 && scatter_lds<4, 4>(nl) <= kLdsBytes) {
        plan_scatter<4, 4>(a, nl, ba.lvl, V_BP44, round, target, out);
    } else if (shape == 2 * 16 + 4 && scatter_lds<2, 4>(nl) <= kLdsBytes) {
        plan_scatter<2, 4>(a, nl, ba.lvl, V_BP24, round, target, out);
    } else if (shape == 1 * 16 + 4 && scatter_lds<1, 4>(nl) <= kLdsBytes) {
        plan_scatter<1, 4>(a, nl, ba.lvl, V_BP14, round, target, out);
    } else if (scatter_lds<2, 8>(nl) <= kLdsBytes) {
        // default tile shapes, measured best on the 512^2 / 720 x 768
        // workload: two rows per wavefront and 8 wavefronts at the two
        // finest levels, four rows and 4 wavefronts on the coarse ones
        if (ba.lvl <= 1)
            plan_scatter<2, 8>(a, nl, ba.lvl, V_BP28, round, target, out);
        else
            plan_scatter<4, 4>(a, nl, ba.lvl, V_BP44, round, target, out);
    } else if (scatter_lds<1, 4>(nl) <= kLdsBytes) {
        // rows longer than about 2400 pixels: fewer rows per workgroup so
        // that they fit in the LDS
        plan_scatter<1, 4>(a, nl, ba.lvl, V_BP14, round, target, out);
    } else {
        plan_scatter<1, 2>(a, nl, ba.lvl, V_BP12, round, target, out);
    }
    if (used) *used = a;
}

hipError_t launch_bp_main(const BpArgs& ba, hipStream_t s, BpOwnArgs& a)
{
    a = own_args(ba);
    const int nl = ba.n >> ba.lvl;
    if (ba.fan.ray) {
        // phases of the scatter: bins P apart are at least P * min_sep apart,
        // 1.25 pixels or more; where rays are denser the gather is used
        const double hl = 2.0 * ba.fan.E / nl;
        const double Pd = std::ceil(1.25 * hl / ba.fan.min_sep);
        if (Pd > kFanScatterMaxP) {
            // view groups: about IMK_FAN_TARGET_WG workgroups, G N_l^2 within
            // the partial-image buffer
            const long long tiles = (long long)((nl + kFanTile - 1) / kFanTile) * ((nl + kFanTile - 1) / kFanTile);
            const long long want = (IMK_FAN_TARGET_WG + tiles - 1) / tiles;
            const long long nv = ba.fan.vb - ba.fan.va;
            const long long room = ba.fan.part_floats / ((long long)nl * nl);
            a.G = (int)std::max(1LL, std::min({want, nv, room, 1024LL}));
            a.nq = a.G;
            hipLaunchKernelGGL(k_bp_fan_gather, dim3((unsigned)tiles, a.G), dim3(256), 0, s, a);
            return hipGetLastError();
        }
        const int phases = (int)std::max(1.0, Pd);
        const size_t m = (size_t)(ba.fan.vb - ba.fan.va) * ba.nd;
        hipLaunchKernelGGL(k_fan_table, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // shape measured on the 512^2 fan workload: one ray per trip; where
        // rays are sparse (P <= 3) 4 wavefronts of 3 owned lines (level 0:
        // 237 against 293 us with 2 lines and 4 rays per trip), else 8
        // wavefronts of 4 lines (level 1: 130 against 168 us with 2 lines
        // and 2 rays); as many wavefronts as fit in the LDS
        const bool sparse = phases <= 3;
        const size_t line = sizeof(float) * (size_t)(nl + 2);
        // lines too long for that many per wavefront in the LDS (grids of
        // more than about 10000 pixels): two per wavefront
        const int rw_want = sparse ? IMK_FAN_ROWS_SPARSE : IMK_FAN_ROWS_DENSE;
        const int rw = (size_t)rw_want * line <= kLdsBytes ? rw_want : 2;
        const int waves = (int)std::max<size_t>(
            1, std::min<size_t>(sparse ? IMK_FAN_SPARSE_WAVES : kFanMaxWaves, kLdsBytes / (rw * line)));
        const int rows = rw * waves;
        const int blocks = (nl + rows - 1) / rows;
        // view groups: about IMK_FAN_SCATTER_WG workgroups (more view groups,
        // shorter workgroups: level 0 of the 512^2 fan workload 424 -> 318 us
        // from 1024 to 4096), 2 G N_l^2 within the partial-image buffer
        const long long want = (IMK_FAN_SCATTER_WG + 2LL * blocks - 1) / (2LL * blocks);
        const long long nv = ba.fan.vb - ba.fan.va;
        const long long room = ba.fan.part_floats / (2LL * nl * nl);
        a.G = (int)std::max(1LL, std::min({want, nv, room, 1024LL}));
        a.nq = 2 * a.G;
        const int lds = (int)(rows * line);
        if (rw == 2) {
            e = allow_lds((const void*)k_bp_fan_scatter<1, 2>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_bp_fan_scatter<1, 2>), dim3(blocks, 2, a.G), dim3(64 * waves), lds, s, a, phases);
        } else if (sparse) {
            e = allow_lds((const void*)k_bp_fan_scatter<1, IMK_FAN_ROWS_SPARSE>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_bp_fan_scatter<1, IMK_FAN_ROWS_SPARSE>), dim3(blocks, 2, a.G), dim3(64 * waves), lds,
                               s, a, phases);
        } else {
            e = allow_lds((const void*)k_bp_fan_scatter<1, IMK_FAN_ROWS_DENSE>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_bp_fan_scatter<1, IMK_FAN_ROWS_DENSE>), dim3(blocks, 2, a.G), dim3(64 * waves), lds,
                               s, a, phases);
        }
        return hipGetLastError();
    }
    Launches r;
    plan_bp_main(ba, 0, r, &a);
    return launch_records(r, s);
}

// Cells per thread of the ordered sums: four (16-byte loads) where the level
// has enough cells to keep the GPU busy that way, else one.
static int sum_cells_per_thread(size_t d) { return d % 4 == 0 && d >= 16384 ? 4 : 1; }

// Slices for about 2^18 threads over d units of work.
static int bp_sum_slices(size_t d, int nq)
{
    int S = 1;  // slices: about 2^18 threads, at most kBpSumMaxSlices, at most nq
    while (S < kBpSumMaxSlices && S < nq && d * (size_t)S < ((size_t)1 << 18)) S *= 2;
    return S;
}

void plan_bp(const BpArgs& ba, int round, Launches& out)
{
    BpOwnArgs a;
    plan_bp_main(ba, round, out, &a);
    const int nl = ba.n >> ba.lvl;
    const size_t d = (size_t)nl * nl;
    SumArgs sa{a, ba.tmp, 0};
    Launch L;
    L.round = round;
    L.block = 1024;
    if (sum_cells_per_thread(d) == 4) {
        sa.S = bp_sum_slices(d / 4, a.nq);
        const size_t cells = 4 * (size_t)(1024 / sa.S);
        L.variant = V_SUM4;
        L.gx = (unsigned)((d + cells - 1) / cells);
    } else {
        sa.S = bp_sum_slices(d, a.nq);
        const size_t cells = 1024 / sa.S;
        L.variant = V_SUM1;
        L.gx = (unsigned)((d + cells - 1) / cells);
    }
    L.set(sa);
    out.push_back(L);
}

void plan_bp_primal(const BpArgs& ba, const PrimalArgs& pr, Launches& out)
{
    BpOwnArgs a;
    plan_bp_main(ba, 0, out, &a);
    const int nl = ba.n >> ba.lvl;
    const size_t d = (size_t)nl * nl;
    SumPrimalArgs sp{a, pr, 0};
    Launch L;
    L.block = 1024;
    if (sum_cells_per_thread(d) == 4) {
        sp.S = bp_sum_slices(d / 4, a.nq);
        const size_t cells = 4 * (size_t)(1024 / sp.S);
        L.variant = V_SUMP4;
        L.gx = (unsigned)((d + cells - 1) / cells);
    } else {
        sp.S = bp_sum_slices(d, a.nq);
        const size_t cells = 1024 / sp.S;
        L.variant = V_SUMP1;
        L.gx = (unsigned)((d + cells - 1) / cells);
    }
    L.set(sp);
    out.push_back(L);
}

bool plan_bp_coarse(const BpArgs* ba, int n, size_t part_floats, bool fused, int round, Launches& out)
{
    // (always succeeds; the result says whether the fused launches were used)
    // each level's tile shape and angle groups, then fewer groups (halving
    // the largest share) until all partial images fit side by side
    BpOwnArgs own[IMASK_MAX_LEVELS];
    int shape[IMASK_MAX_LEVELS], nb[IMASK_MAX_LEVELS], block[IMASK_MAX_LEVELS], lds[IMASK_MAX_LEVELS];
    for (int t = 0; t < n; ++t) {
        Launches tmp;
        plan_bp_main(ba[t], 0, tmp, &own[t]);
        shape[t] = tmp.back().variant;
        nb[t] = (int)tmp.back().gx;
        block[t] = tmp.back().block;
        lds[t] = tmp.back().lds;
        // the fused launches exist for the 2x8 and 4x4 tiles; other tiles
        // run as records of their own with the same partial-image layout
        if (shape[t] != V_BP28 && shape[t] != V_BP44) fused = false;
    }
    auto share = [&](int t) { return (size_t)own[t].nq * (size_t)(ba[t].n >> ba[t].lvl) * (ba[t].n >> ba[t].lvl); };
    for (;;) {
        size_t total = 0;
        int big = 0;
        for (int t = 0; t < n; ++t) {
            total += share(t);
            if (share(t) > share(big)) big = t;
        }
        if (total <= part_floats || own[big].G == 1) break;
        own[big].G = std::max(1, own[big].G / 2);
        own[big].nq = 2 * own[big].G;
    }
    size_t off = 0;
    for (int t = 0; t < n; ++t) {
        own[t].part = ba[t].part + off;
        off += share(t);
    }
    if (!fused) {  // the same transposes and sums as records of their own (disjoint partial images)
        for (int t = 0; t < n; ++t) {
            Launch L;
            L.variant = shape[t];
            L.round = round;
            L.gx = (unsigned)nb[t];
            L.gy = (unsigned)(2 * own[t].G);
            L.block = block[t];
            L.lds = lds[t];
            L.set(own[t]);
            out.push_back(L);
        }
    }
    for (int v : {V_BP28, V_BP44}) {
        if (!fused) break;
        BpMultiArgs m{};
        Launch L;
        L.variant = v == V_BP28 ? V_BP_MULTI28 : V_BP_MULTI44;
        L.block = v == V_BP28 ? 512 : 256;
        for (int t = 0; t < n; ++t) {
            if (shape[t] != v) continue;
            const int nl = ba[t].n >> ba[t].lvl;
            m.t[m.n] = own[t];
            m.gx[m.n] = nb[t];
            m.start[m.n + 1] = m.start[m.n] + nb[t] * 2 * own[t].G;
            L.lds = std::max(L.lds, (int)(v == V_BP28 ? scatter_lds<2, 8>(nl) : scatter_lds<4, 4>(nl)));
            ++m.n;
        }
        if (m.n == 0) continue;
        L.gx = (unsigned)m.start[m.n];
        L.set(m);
        out.push_back(L);
    }
    SumMultiArgs sm{};
    sm.n = n;
    for (int t = 0; t < n; ++t) {
        const int nl = ba[t].n >> ba[t].lvl;
        const size_t d = (size_t)nl * nl;
        SumArgs sa{own[t], ba[t].tmp, 0};
        size_t cells;
        if (sum_cells_per_thread(d) == 4) {
            sa.S = bp_sum_slices(d / 4, own[t].nq);
            cells = 4 * (size_t)(1024 / sa.S);
            sm.v[t] = 4;
        } else {
            sa.S = bp_sum_slices(d, own[t].nq);
            cells = 1024 / sa.S;
            sm.v[t] = 1;
        }
        sm.t[t] = sa;
        sm.start[t + 1] = sm.start[t] + (int)((d + cells - 1) / cells);
        if (!fused) {
            Launch L;
            L.variant = sm.v[t] == 4 ? V_SUM4 : V_SUM1;
            L.round = round;
            L.block = 1024;
            L.gx = (unsigned)((d + cells - 1) / cells);
            L.set(sa);
            out.push_back(L);
        }
    }
    if (!fused) return false;
    Launch L;
    L.variant = V_SUM_MULTI;
    L.block = 1024;
    L.gx = (unsigned)sm.start[n];
    L.set(sm);
    out.push_back(L);
    return true;
}

// The ordered sum of the fan-beam transposes' partial images (and the
// prolongation of either beam's result when asked for).
static hipError_t launch_sum_after(const BpArgs& ba, const BpOwnArgs& a, hipStream_t s)
{
    const int nl = ba.n >> ba.lvl;
    const size_t d = (size_t)nl * nl;
    if (sum_cells_per_thread(d) == 4) {
        const int S = bp_sum_slices(d / 4, a.nq);
        const size_t cells = 4 * (size_t)(1024 / S);
        hipLaunchKernelGGL(k_bp_sum<4>, dim3((unsigned)((d + cells - 1) / cells)), dim3(1024), 0, s, a, ba.tmp, S);
    } else {
        const int S = bp_sum_slices(d, a.nq);
        const size_t cells = 1024 / S;
        hipLaunchKernelGGL(k_bp_sum<1>, dim3((unsigned)((d + cells - 1) / cells)), dim3(1024), 0, s, a, ba.tmp, S);
    }
    return hipGetLastError();
}

hipError_t launch_bp(const BpArgs& ba, hipStream_t s)
{
    hipError_t e;
    if (ba.fan.ray) {
        BpOwnArgs a;
        e = launch_bp_main(ba, s, a);
        if (e != hipSuccess) return e;
        e = launch_sum_after(ba, a, s);
    } else {
        Launches r;
        plan_bp(ba, 0, r);
        e = launch_records(r, s);
    }
    if (e != hipSuccess || !ba.prolong) return e;
    const size_t fine = (size_t)ba.n * ba.n;
    hipLaunchKernelGGL(k_prolong_acc, dim3((unsigned)((fine + 255) / 256)), dim3(256), 0, s, (const float*)ba.tmp,
                       ba.out, ba.n, ba.lvl, ba.accumulate);
    return hipGetLastError();
}

hipError_t launch_bp_primal(const BpArgs& ba, const PrimalArgs& pr, hipStream_t s)
{
    if (!ba.fan.ray) {
        Launches r;
        plan_bp_primal(ba, pr, r);
        return launch_records(r, s);
    }
    BpOwnArgs a;
    hipError_t e = launch_bp_main(ba, s, a);
    if (e != hipSuccess) return e;
    const int nl = ba.n >> ba.lvl;
    const size_t d = (size_t)nl * nl;
    if (sum_cells_per_thread(d) == 4) {
        const int S = bp_sum_slices(d / 4, a.nq);
        const size_t cells = 4 * (size_t)(1024 / S);
        hipLaunchKernelGGL(k_bp_sum_primal<4>, dim3((unsigned)((d + cells - 1) / cells)), dim3(1024), 0, s, a, S, pr);
    } else {
        const int S = bp_sum_slices(d, a.nq);
        const size_t cells = 1024 / S;
        hipLaunchKernelGGL(k_bp_sum_primal<1>, dim3((unsigned)((d + cells - 1) / cells)), dim3(1024), 0, s, a, S, pr);
    }
    return hipGetLastError();
}

bool sum_primal_tile_fits(const PrimalArgs& pr) { return pr.n % 32 == 0 && pr.pyr_levels <= 5; }

void plan_sum_primal_tile(const BpOwnArgs& a, const PrimalArgs& pr, Launches& out)
{
    // 32 x 32 tiles (whole 128-byte rows of every partial image, 16-byte
    // loads); sum_primal_tile_fits holds
    PrimalArgs p = pr;
    p.T = 32;
    Launch L;
    L.variant = V_SUMPT;
    const int tiles = p.n / p.T;
    L.gx = (unsigned)(tiles * tiles);
    L.block = kSumTileThreads;
    static_assert(kSumTileThreads == kSumTileSlices * 32 * 32 / 4, "four pixels per thread per slice");
    L.lds = (int)((2 + kSumTileSlices) * 32 * 32 * sizeof(float));  // pyramid, then the slice sums
    L.set(SumTileArgs{a, p});
    out.push_back(L);
}

void merge_reduce_into_transpose(Launches& out)
{
    size_t r = out.size(), t = out.size();
    for (size_t q = 0; q < out.size(); ++q)
        if (out[q].variant == V_RED4 || out[q].variant == V_RED1) {
            r = q;
            break;
        }
    for (size_t q = r + 1; q < out.size(); ++q) {
        const int v = out[q].variant;
        if (v == V_BP28 || v == V_BP44 || v == V_BP14 || v == V_BP12 || v == V_BP24) {
            t = q;
            break;
        }
    }
    if (r >= out.size() || t >= out.size() || out[t].gz != 1) return;
    const Launch& red = out[r];
    Launch& tr = out[t];
    BpRedArgs m{};
    m.b = tr.get<BpOwnArgs>();
    m.f = red.get<FwdArgs>();
    m.bgx = (int)tr.gx;
    m.nbp = (int)(tr.gx * tr.gy);
    // the reduce's grid-stride loop covers the sinogram with any block size
    m.nred = (int)red.gx;
    m.red4 = red.variant == V_RED4;
    const int v = tr.variant;
    tr.variant = v == V_BP28 ? V_BPRED28 : v == V_BP44 ? V_BPRED44 : v == V_BP14 ? V_BPRED14
                 : v == V_BP12 ? V_BPRED12 : V_BPRED24;
    tr.gx = (unsigned)(m.nbp + m.nred);
    tr.gy = 1;
    tr.set(m);
    out.erase(out.begin() + (long)r);
}

void merge_forward_into_transpose(Launches& out)
{
    size_t f = out.size(), t = out.size();
    for (size_t q = 0; q < out.size(); ++q)
        if (out[q].variant == V_FWD_BAND && out[q].get<FwdBandArgs>().dual) {
            f = q;
            break;
        }
    for (size_t q = f + 1; q < out.size(); ++q) {
        const int v = out[q].variant;
        if (v == V_RED4 || v == V_RED1) return;  // a reduce follows: the forward has several bands
        if (v == V_BP28 || v == V_BP44 || v == V_BP14 || v == V_BP12 || v == V_BP24) {
            t = q;
            break;
        }
    }
    if (f >= out.size() || t >= out.size() || out[t].gz != 1 || out[f].gx != 1) return;
    const Launch& fw = out[f];
    Launch& tr = out[t];
    BpFwdArgs m{};
    m.b = tr.get<BpOwnArgs>();
    m.f = fw.get<FwdBandArgs>();
    // the forward's groups sized for the transpose's block: about as many
    // rays per thread as with 1024 threads
    const int scale = std::max(1, 1024 / (int)tr.block);
    const int apg = std::max(1, m.f.apg / scale);
    m.f.apg = apg;
    m.f.groups_row = (m.f.split.nrow + apg - 1) / apg;
    m.f.groups_col = (m.f.split.ncol + apg - 1) / apg;
    m.bgx = (int)tr.gx;
    m.nbp = (int)(tr.gx * tr.gy);
    m.fgx = 1;
    m.nfwd = m.f.groups_row + m.f.groups_col;
    const int v = tr.variant;
    tr.variant = v == V_BP28 ? V_BPFWD28 : v == V_BP44 ? V_BPFWD44 : v == V_BP14 ? V_BPFWD14
                 : v == V_BP12 ? V_BPFWD12 : V_BPFWD24;
    tr.gx = (unsigned)(m.nbp + m.nfwd);
    tr.gy = 1;
    tr.lds = std::max(tr.lds, fw.lds);
    tr.set(m);
    out.erase(out.begin() + (long)f);
}

void plan_primal(const PrimalArgs& a, Launches& out)
{
    Launch L;
    L.variant = V_PRIMAL;
    const int tiles = a.n / a.T;
    const bool paper_full = (a.kidx == 0 && a.full_mode == IMASK_FULL_PAPER && a.r > 1);
    L.gx = (unsigned)(tiles * tiles);
    L.block = 256;
    L.lds = paper_full ? (int)pyramid_bytes(a.T, a.pyr_levels) : 0;
    L.set(a);
    out.push_back(L);
}

hipError_t launch_primal(const PrimalArgs& a, hipStream_t s)
{
    Launches r;
    plan_primal(a, r);
    return launch_records(r, s);
}

// Kernel of each variant (the single-problem form).
static const void* variant_kernel(int v)
{
    switch (v) {
    case V_PREP: return (const void*)k_prep;
    case V_FWD_BAND: return (const void*)k_fwd_band;
    case V_FWD_DIRECT: return (const void*)k_fwd_direct;
    case V_RED4: return (const void*)k_fwd_reduce4;
    case V_RED1: return (const void*)k_fwd_reduce;
    case V_BP28: return (const void*)k_bp_own<2, 8>;
    case V_BP44: return (const void*)k_bp_own<4, 4>;
    case V_BP14: return (const void*)k_bp_own<1, 4>;
    case V_BP12: return (const void*)k_bp_own<1, 2>;
    case V_BP24: return (const void*)k_bp_own<2, 4>;
    case V_SUM4: return (const void*)k_bp_sum<4>;
    case V_SUM1: return (const void*)k_bp_sum<1>;
    case V_SUMP4: return (const void*)k_bp_sum_primal<4>;
    case V_SUMP1: return (const void*)k_bp_sum_primal<1>;
    case V_PRIMAL: return (const void*)k_primal;
    case V_SUMPT: return (const void*)k_sum_primal_tile;
    case V_FWD_MULTI: return (const void*)k_fwd_band_multi;
    case V_BP_MULTI28: return (const void*)k_bp_own_multi<2, 8>;
    case V_BP_MULTI44: return (const void*)k_bp_own_multi<4, 4>;
    case V_SUM_MULTI: return (const void*)k_bp_sum_multi;
    case V_BPRED28: return (const void*)k_bp_red<2, 8>;
    case V_BPRED44: return (const void*)k_bp_red<4, 4>;
    case V_BPRED14: return (const void*)k_bp_red<1, 4>;
    case V_BPRED12: return (const void*)k_bp_red<1, 2>;
    case V_BPRED24: return (const void*)k_bp_red<2, 4>;
    case V_BPFWD28: return (const void*)k_bp_fwd<2, 8>;
    case V_BPFWD44: return (const void*)k_bp_fwd<4, 4>;
    case V_BPFWD14: return (const void*)k_bp_fwd<1, 4>;
    case V_BPFWD12: return (const void*)k_bp_fwd<1, 2>;
    case V_BPFWD24: return (const void*)k_bp_fwd<2, 4>;
    default: return nullptr;
    }
}

hipError_t launch_records(const Launches& recs, hipStream_t s)
{
    for (const Launch& L : recs) {
        const dim3 grid(L.gx, L.gy, L.gz), block(L.block);
        const hipError_t e0 = allow_lds(variant_kernel(L.variant), L.lds);
        if (e0 != hipSuccess) return e0;
        switch (L.variant) {
        case V_PREP: hipLaunchKernelGGL(k_prep, grid, block, L.lds, s, L.get<PrepArgs>()); break;
        case V_FWD_BAND: hipLaunchKernelGGL(k_fwd_band, grid, block, L.lds, s, L.get<FwdBandArgs>()); break;
        case V_FWD_DIRECT: hipLaunchKernelGGL(k_fwd_direct, grid, block, L.lds, s, L.get<FwdBandArgs>()); break;
        case V_RED4: hipLaunchKernelGGL(k_fwd_reduce4, grid, block, L.lds, s, L.get<FwdArgs>()); break;
        case V_RED1: hipLaunchKernelGGL(k_fwd_reduce, grid, block, L.lds, s, L.get<FwdArgs>()); break;
        case V_BP28: hipLaunchKernelGGL((k_bp_own<2, 8>), grid, block, L.lds, s, L.get<BpOwnArgs>()); break;
        case V_BP44: hipLaunchKernelGGL((k_bp_own<4, 4>), grid, block, L.lds, s, L.get<BpOwnArgs>()); break;
        case V_BP14: hipLaunchKernelGGL((k_bp_own<1, 4>), grid, block, L.lds, s, L.get<BpOwnArgs>()); break;
        case V_BP12: hipLaunchKernelGGL((k_bp_own<1, 2>), grid, block, L.lds, s, L.get<BpOwnArgs>()); break;
        case V_BP24: hipLaunchKernelGGL((k_bp_own<2, 4>), grid, block, L.lds, s, L.get<BpOwnArgs>()); break;
        case V_SUM4: {
            const SumArgs& a = L.get<SumArgs>();
            hipLaunchKernelGGL(k_bp_sum<4>, grid, block, L.lds, s, a.a, a.tmp, a.S);
            break;
        }
        case V_SUM1: {
            const SumArgs& a = L.get<SumArgs>();
            hipLaunchKernelGGL(k_bp_sum<1>, grid, block, L.lds, s, a.a, a.tmp, a.S);
            break;
        }
        case V_SUMP4: {
            const SumPrimalArgs& a = L.get<SumPrimalArgs>();
            hipLaunchKernelGGL(k_bp_sum_primal<4>, grid, block, L.lds, s, a.a, a.S, a.p);
            break;
        }
        case V_SUMP1: {
            const SumPrimalArgs& a = L.get<SumPrimalArgs>();
            hipLaunchKernelGGL(k_bp_sum_primal<1>, grid, block, L.lds, s, a.a, a.S, a.p);
            break;
        }
        case V_PRIMAL: hipLaunchKernelGGL(k_primal, grid, block, L.lds, s, L.get<PrimalArgs>()); break;
        case V_SUMPT: hipLaunchKernelGGL(k_sum_primal_tile, grid, block, L.lds, s, L.get<SumTileArgs>()); break;
        case V_FWD_MULTI: hipLaunchKernelGGL(k_fwd_band_multi, grid, block, L.lds, s, L.get<FwdMultiArgs>()); break;
        case V_BP_MULTI28:
            hipLaunchKernelGGL((k_bp_own_multi<2, 8>), grid, block, L.lds, s, L.get<BpMultiArgs>());
            break;
        case V_BP_MULTI44:
            hipLaunchKernelGGL((k_bp_own_multi<4, 4>), grid, block, L.lds, s, L.get<BpMultiArgs>());
            break;
        case V_SUM_MULTI: hipLaunchKernelGGL(k_bp_sum_multi, grid, block, L.lds, s, L.get<SumMultiArgs>()); break;
        case V_BPRED28: hipLaunchKernelGGL((k_bp_red<2, 8>), grid, block, L.lds, s, L.get<BpRedArgs>()); break;
        case V_BPRED44: hipLaunchKernelGGL((k_bp_red<4, 4>), grid, block, L.lds, s, L.get<BpRedArgs>()); break;
        case V_BPRED14: hipLaunchKernelGGL((k_bp_red<1, 4>), grid, block, L.lds, s, L.get<BpRedArgs>()); break;
        case V_BPRED12: hipLaunchKernelGGL((k_bp_red<1, 2>), grid, block, L.lds, s, L.get<BpRedArgs>()); break;
        case V_BPRED24: hipLaunchKernelGGL((k_bp_red<2, 4>), grid, block, L.lds, s, L.get<BpRedArgs>()); break;
        case V_BPFWD28: hipLaunchKernelGGL((k_bp_fwd<2, 8>), grid, block, L.lds, s, L.get<BpFwdArgs>()); break;
        case V_BPFWD44: hipLaunchKernelGGL((k_bp_fwd<4, 4>), grid, block, L.lds, s, L.get<BpFwdArgs>()); break;
        case V_BPFWD14: hipLaunchKernelGGL((k_bp_fwd<1, 4>), grid, block, L.lds, s, L.get<BpFwdArgs>()); break;
        case V_BPFWD12: hipLaunchKernelGGL((k_bp_fwd<1, 2>), grid, block, L.lds, s, L.get<BpFwdArgs>()); break;
        case V_BPFWD24: hipLaunchKernelGGL((k_bp_fwd<2, 4>), grid, block, L.lds, s, L.get<BpFwdArgs>()); break;
        default: return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tv(const TvArgs& a, hipStream_t s)
{
    const int R = kTvTile + 2 * a.J;
    const size_t sh = (size_t)3 * R * R * sizeof(float);
    const int tiles = (a.n + kTvTile - 1) / kTvTile;
    const hipError_t e = allow_lds((const void*)k_tv, (int)sh);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tv, dim3(tiles * tiles), dim3(kTvThreads), sh, s, a);
    return hipGetLastError();
}

hipError_t launch_tvd(const TvdArgs& a, hipStream_t s)
{
    const int R = kTvTile + 2 * (a.J + 1);
    const size_t sh = (size_t)3 * R * R * sizeof(float);
    const int tiles = (a.n + kTvTile - 1) / kTvTile;
    const hipError_t e = allow_lds((const void*)k_tvd, (int)sh);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tvd, dim3(tiles * tiles), dim3(kTvThreads), sh, s, a);
    return hipGetLastError();
}

hipError_t launch_prolong(const float* in, float* out, int n, int lvl, float coef, hipStream_t s)
{
    const size_t count = (size_t)n * n;
    hipLaunchKernelGGL(k_prolong, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, in, out, n, lvl, coef);
    return hipGetLastError();
}

hipError_t launch_project_block(const float* in, float* out, int n, int lvl, hipStream_t s)
{
    const size_t count = (size_t)n * n;
    hipLaunchKernelGGL(k_project_block, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, in, out, n, lvl);
    return hipGetLastError();
}

}  // namespace imk

namespace imk {

static unsigned vec_blocks(size_t n)
{
    size_t b = (n + 255) / 256;
    return (unsigned)std::max<size_t>(1, std::min<size_t>(b, 2048));
}

hipError_t launch_axpy(float* y, const float* x, float a, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, dim3(vec_blocks(n)), dim3(256), 0, s, y, x, a, n);
    return hipGetLastError();
}

hipError_t launch_scale(float* x, float a, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(vec_blocks(n)), dim3(256), 0, s, x, a, n);
    return hipGetLastError();
}

hipError_t launch_fill_random(float* x, size_t n, unsigned long long seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_random, dim3(vec_blocks(n)), dim3(256), 0, s, x, n, seed);
    return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, size_t n, double* part, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, a, b, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kDotBlocks), 0, s, (const double*)part, out);
    return hipGetLastError();
}

}  // namespace imk

// ------------------------------------------------- batched steps (many problems)
//
// A batch holds, for every problem, sketch index and parity of the state's
// ping-pong buffers, the launch records of that step (the same records the
// single-problem launchers run).  Each step is one plan kernel, one
// persistent launch per (kernel variant, round) over the work items of every
// problem that needs that variant this step, and one advance kernel; the
// sketch index is drawn on the device, so the launches of a step do not
// depend on the draw and a captured step replays as it is.

namespace imk {
namespace {

// SplitMix64 output k + 1 of the stream at state0 (Steele, Lea & Flood
// 2014, counter form), as the host draw computes it.
__device__ __forceinline__ unsigned long long batch_mix(unsigned long long state0, unsigned long long k)
{
    unsigned long long z = state0 + (k + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Draws each active problem's sketch index, selects its records and forms,
// per stage slot (variant, round), the running offsets of the problems' work
// items and a list of segments, one per record of that slot (its index and
// its first item), which the stage kernels search.
__global__ void __launch_bounds__(1024) k_batch_plan(BatchView bv)
{
    const int n = bv.n;
    const int slots = kNumVariants * kRounds;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const BatchProb& pb = bv.prob[q];
        int sl = -1;
        if (pb.k < pb.k_stop) {
            const unsigned long long u = batch_mix(pb.stream_state, pb.k) >> 32;
            int j = 0;
            while (j < pb.r - 1 && u >= pb.thr[j]) ++j;
            sl = j * 2 + pb.cur;
        }
        bv.sel[q] = sl;
    }
    __syncthreads();
    // per (problem, stage slot): its items and records, at the problem's
    // place in the work order (largest problems first, so their long items
    // start early and the short ones fill the tail)
    for (int idx = threadIdx.x; idx < n * slots; idx += blockDim.x) {
        const int q = idx / slots, vr = idx - q * slots;
        const int sl = bv.sel[q];
        const size_t base = ((size_t)q * bv.r_max * 2 + (sl >= 0 ? sl : 0)) * slots;
        const size_t at = (size_t)vr * (n + 1) + bv.rank[q] + 1;
        bv.off[at] = sl >= 0 ? bv.items[base + vr] : 0;
        bv.segc[at] = sl >= 0 ? bv.nsegs[base + vr] : 0;
    }
    __syncthreads();
    // running sums in registers (a chain through memory would wait on every
    // store it just made)
    for (int vr = threadIdx.x; vr < slots; vr += blockDim.x) {
        int* o = bv.off + (size_t)vr * (n + 1);
        int* c = bv.segc + (size_t)vr * (n + 1);
        int so = 0, sc = 0;
        o[0] = 0;
        c[0] = 0;
        for (int q = 0; q < n; ++q) {
            so += o[q + 1];
            sc += c[q + 1];
            o[q + 1] = so;
            c[q + 1] = sc;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        bv.seg_off[0] = 0;
        for (int vr = 0; vr < slots; ++vr) {
            acc += bv.segc[(size_t)vr * (n + 1) + n];
            bv.seg_off[vr + 1] = acc;
        }
    }
    __syncthreads();
    // one segment per record of each active problem: its place among the
    // slot's segments and its first item (the counts of earlier records of
    // the same slot are stored with the record)
    for (int idx = threadIdx.x; idx < n * kMaxRec; idx += blockDim.x) {
        const int q = idx / kMaxRec, j = idx - q * kMaxRec;
        const int sl = bv.sel[q];
        if (sl < 0) continue;
        const size_t sq = (size_t)q * bv.r_max * 2 + sl;
        if (j >= bv.nrec[sq]) continue;
        const BatchRec& rc = bv.rec[sq * kMaxRec + j];
        const int vr = rc.variant * kRounds + rc.round;
        const int rq = bv.rank[q];
        const int pos = bv.seg_off[vr] + bv.segc[(size_t)vr * (n + 1) + rq] + rc.ord;
        bv.seg[2 * pos] = (int)(sq * kMaxRec + j);
        bv.seg[2 * pos + 1] = bv.off[(size_t)vr * (n + 1) + rq] + rc.ibefore;
    }
}

// k += 1, parity flip and the sketch's epochs for every problem that stepped.
__global__ void k_batch_advance(BatchView bv)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= bv.n) return;
    const int sl = bv.sel[q];
    if (sl < 0) return;
    BatchProb& pb = bv.prob[q];
    pb.epochs += pb.cost[sl >> 1];
    pb.k += 1ULL;
    pb.cur ^= 1;
}

// The argument block of an item as a value every lane holds alike: each word
// read from LDS goes through readfirstlane, so the compiler keeps the
// arguments (and what the body derives from them) in scalar registers, as
// it does for a kernel's own arguments (read in place from LDS, they are
// per-lane values to it: the transpose's inner loop then issued 60% more
// VALU instructions).  Used where the block has no array the body indexes
// at run time; such a copy would live in scratch memory.
template <class T>
__device__ __forceinline__ T uniform_args(const unsigned char* lds)
{
    static_assert(sizeof(T) % 4 == 0, "argument blocks are whole words");
    constexpr int nw = (int)(sizeof(T) / 4);
    int w[nw];
#pragma unroll
    for (int i = 0; i < nw; ++i) w[i] = __builtin_amdgcn_readfirstlane(reinterpret_cast<const int*>(lds)[i]);
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

template <int V>
__device__ __forceinline__ void batch_body(const unsigned char* args, const Blk& bk, float* smem)
{
    if constexpr (V == V_PREP) {
        prep_body(*reinterpret_cast<const PrepArgs*>(args), bk, smem);
    } else if constexpr (V == V_FWD_BAND) {
        fwd_band_body(*reinterpret_cast<const FwdBandArgs*>(args), bk, smem);
    } else if constexpr (V == V_FWD_DIRECT) {
        fwd_direct_body(*reinterpret_cast<const FwdBandArgs*>(args), bk);
    } else if constexpr (V == V_RED4) {
        fwd_reduce4_body(*reinterpret_cast<const FwdArgs*>(args), bk);
    } else if constexpr (V == V_RED1) {
        fwd_reduce_body(*reinterpret_cast<const FwdArgs*>(args), bk);
    } else if constexpr (V == V_BP28) {
        bp_own_body<2, 8>(uniform_args<BpOwnArgs>(args), bk, smem);
    } else if constexpr (V == V_BP44) {
        bp_own_body<4, 4>(uniform_args<BpOwnArgs>(args), bk, smem);
    } else if constexpr (V == V_BP14) {
        bp_own_body<1, 4>(uniform_args<BpOwnArgs>(args), bk, smem);
    } else if constexpr (V == V_BP12) {
        bp_own_body<1, 2>(uniform_args<BpOwnArgs>(args), bk, smem);
    } else if constexpr (V == V_BP24) {
        bp_own_body<2, 4>(uniform_args<BpOwnArgs>(args), bk, smem);
    } else if constexpr (V == V_SUM4 || V == V_SUM1) {
        const SumArgs a = uniform_args<SumArgs>(args);
        bp_sum_body<V == V_SUM4 ? 4 : 1>(a.a, a.tmp, a.S, bk);
    } else if constexpr (V == V_SUMP4 || V == V_SUMP1) {
        const SumPrimalArgs& a = *reinterpret_cast<const SumPrimalArgs*>(args);
        bp_sum_primal_body<V == V_SUMP4 ? 4 : 1>(a.a, a.S, a.p, bk);
    } else if constexpr (V == V_SUMPT) {
        const SumTileArgs& a = *reinterpret_cast<const SumTileArgs*>(args);
        sum_primal_tile_body(a.a, a.p, bk, smem);
    } else {
        primal_body(*reinterpret_cast<const PrimalArgs*>(args), bk, smem);
    }
}

static_assert(sizeof(PrepArgs) <= kBlobBytes && sizeof(FwdBandArgs) <= kBlobBytes && sizeof(FwdArgs) <= kBlobBytes &&
                  sizeof(BpOwnArgs) <= kBlobBytes && sizeof(SumArgs) <= kBlobBytes &&
                  sizeof(SumPrimalArgs) <= kBlobBytes && sizeof(SumTileArgs) <= kBlobBytes &&
                  sizeof(PrimalArgs) <= kBlobBytes,
              "a batched variant's argument block fits its slot");

// Threads per workgroup of each variant (those of its single-problem kernel).
template <int V>
constexpr int kVariantThreads = (V == V_FWD_BAND || V == V_SUM4 || V == V_SUM1 || V == V_SUMP4 || V == V_SUMP1 ||
                                  V == V_SUMPT)
                                     ? 1024
                                : V == V_BP28                                                                    ? 512
                                : V == V_BP12                                                                    ? 128
                                                                                                                 : 256;

// Persistent launch of variant V, round `round`: workgroup w takes items
// w, w + grid, ... of the step's list; an item is one workgroup of one
// problem's launch, found from the offsets by binary search.  The argument
// block is staged in LDS, where every thread reads it.
constexpr int kSegLds = 64;  // segment starts a stage kernel keeps in LDS (more: searched in memory); small, so
                             // that the static LDS leaves the large transposes four workgroups per CU

template <int V>
__global__ void __launch_bounds__(kVariantThreads<V>) k_batch(BatchView bv, int round, int lds_avail)
{
    extern __shared__ float smem[];
    __shared__ __attribute__((aligned(16))) unsigned char s_args[kBlobBytes];
    __shared__ int s_start[kSegLds];
    const int n = bv.n;
    const int vr = V * kRounds + round;
    const int total = bv.off[(size_t)vr * (n + 1) + n];
    const int s0 = bv.seg_off[vr], nseg = bv.seg_off[vr + 1] - s0;
    const int* seg = bv.seg + 2 * (size_t)s0;
    const bool in_lds = nseg <= kSegLds;
    if (in_lds) {
        for (int t = threadIdx.x; t < nseg; t += blockDim.x) s_start[t] = seg[2 * t + 1];
        __syncthreads();
    }
    // the record of an item and the item's place in its launch
    auto find = [&](int item, int& local) -> BatchRec {
        int lo = 0, hi = nseg;  // start[lo] <= item < start[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            const int st = in_lds ? s_start[mid] : seg[2 * mid + 1];
            if (st <= item) lo = mid; else hi = mid;
        }
        const int sgi = __builtin_amdgcn_readfirstlane(lo);
        local = item - seg[2 * sgi + 1];
        return bv.rec[seg[2 * sgi]];
    };
    static_assert(kBlobBytes / 16 <= 128, "one 16-byte word of an argument block per thread");
    const bool loader = threadIdx.x < kBlobBytes / 16;
    // threads below kBlobBytes / 16 hold one word of the next item's
    // argument block, read while the current item runs
    uint4 next = {0u, 0u, 0u, 0u};
    int item = blockIdx.x, local = 0;
    BatchRec rc{};
    if (item < total) {
        rc = find(item, local);
        if (loader) next = reinterpret_cast<const uint4*>(bv.blobs + (size_t)rc.blob * kBlobBytes)[threadIdx.x];
    }
    while (item < total) {
        if (loader) reinterpret_cast<uint4*>(s_args)[threadIdx.x] = next;
        __syncthreads();
        const int item2 = item + gridDim.x;
        int local2 = 0;
        BatchRec rc2{};
        if (item2 < total) {
            rc2 = find(item2, local2);
            if (loader) next = reinterpret_cast<const uint4*>(bv.blobs + (size_t)rc2.blob * kBlobBytes)[threadIdx.x];
        }
        // always true: the segments cover exactly these items, and the
        // launch reserves the LDS of its largest record
        if (rc.variant == V && local < rc.items && rc.lds <= lds_avail) {
            Blk bk;
            bk.x = local % rc.gx;
            const int t2 = local / rc.gx;
            bk.y = t2 % rc.gy;
            bk.z = t2 / rc.gy;
            bk.gx = rc.gx;
            batch_body<V>(s_args, bk, smem);
        }
        __syncthreads();  // the next item rewrites the arguments and the LDS
        item = item2;
        local = local2;
        rc = rc2;
    }
}

}  // namespace

int variant_threads(int v)
{
    switch (v) {
    case V_FWD_BAND: case V_SUM4: case V_SUM1: case V_SUMP4: case V_SUMP1: case V_SUMPT: return 1024;
    case V_BP28: return 512;
    case V_BP12: return 128;
    default: return 256;
    }
}

template <int V>
static const void* batch_kernel() { return (const void*)k_batch<V>; }

static const void* batch_kernel_of(int v)
{
    switch (v) {
    case V_PREP: return batch_kernel<V_PREP>();
    case V_FWD_BAND: return batch_kernel<V_FWD_BAND>();
    case V_FWD_DIRECT: return batch_kernel<V_FWD_DIRECT>();
    case V_RED4: return batch_kernel<V_RED4>();
    case V_RED1: return batch_kernel<V_RED1>();
    case V_BP28: return batch_kernel<V_BP28>();
    case V_BP44: return batch_kernel<V_BP44>();
    case V_BP14: return batch_kernel<V_BP14>();
    case V_BP12: return batch_kernel<V_BP12>();
    case V_BP24: return batch_kernel<V_BP24>();
    case V_SUM4: return batch_kernel<V_SUM4>();
    case V_SUM1: return batch_kernel<V_SUM1>();
    case V_SUMP4: return batch_kernel<V_SUMP4>();
    case V_SUMP1: return batch_kernel<V_SUMP1>();
    case V_PRIMAL: return batch_kernel<V_PRIMAL>();
    case V_SUMPT: return batch_kernel<V_SUMPT>();
    default: return nullptr;
    }
}

// Static LDS of a batched variant: the staged argument block and segment
// starts, plus the ordered sums' reduction arrays.
size_t variant_static_lds(int v)
{
    size_t s = kBlobBytes + kSegLds * sizeof(int);
    if (v == V_SUM4) s += 1024 * 4 * sizeof(float);
    if (v == V_SUM1) s += 1024 * sizeof(float);
    if (v == V_SUMP4) s += 3 * 1024 * 4 * sizeof(float);
    if (v == V_SUMP1) s += 3 * 1024 * sizeof(float);
    return s;
}

hipError_t batch_allow_lds(int v, int lds) { return allow_lds(batch_kernel_of(v), lds); }

hipError_t launch_batch_plan(const BatchView& bv, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, s, bv);
    return hipGetLastError();
}

hipError_t launch_batch_advance(const BatchView& bv, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_advance, dim3((unsigned)((bv.n + 255) / 256)), dim3(256), 0, s, bv);
    return hipGetLastError();
}

hipError_t launch_batch_stage(int v, int round, const BatchView& bv, unsigned grid, int lds, hipStream_t s)
{
    const dim3 g(grid);
    switch (v) {
    case V_PREP: hipLaunchKernelGGL(k_batch<V_PREP>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_FWD_BAND: hipLaunchKernelGGL(k_batch<V_FWD_BAND>, g, dim3(1024), lds, s, bv, round, lds); break;
    case V_FWD_DIRECT: hipLaunchKernelGGL(k_batch<V_FWD_DIRECT>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_RED4: hipLaunchKernelGGL(k_batch<V_RED4>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_RED1: hipLaunchKernelGGL(k_batch<V_RED1>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_BP28: hipLaunchKernelGGL(k_batch<V_BP28>, g, dim3(512), lds, s, bv, round, lds); break;
    case V_BP44: hipLaunchKernelGGL(k_batch<V_BP44>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_BP14: hipLaunchKernelGGL(k_batch<V_BP14>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_BP12: hipLaunchKernelGGL(k_batch<V_BP12>, g, dim3(128), lds, s, bv, round, lds); break;
    case V_BP24: hipLaunchKernelGGL(k_batch<V_BP24>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_SUM4: hipLaunchKernelGGL(k_batch<V_SUM4>, g, dim3(1024), lds, s, bv, round, lds); break;
    case V_SUM1: hipLaunchKernelGGL(k_batch<V_SUM1>, g, dim3(1024), lds, s, bv, round, lds); break;
    case V_SUMP4: hipLaunchKernelGGL(k_batch<V_SUMP4>, g, dim3(1024), lds, s, bv, round, lds); break;
    case V_SUMP1: hipLaunchKernelGGL(k_batch<V_SUMP1>, g, dim3(1024), lds, s, bv, round, lds); break;
    case V_PRIMAL: hipLaunchKernelGGL(k_batch<V_PRIMAL>, g, dim3(256), lds, s, bv, round, lds); break;
    case V_SUMPT: hipLaunchKernelGGL(k_batch<V_SUMPT>, g, dim3(1024), lds, s, bv, round, lds); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace imk
