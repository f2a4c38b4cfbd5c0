// kernels.hip - gfx950 kernels of the ImaSk hot path.
//
// Projector pair (Sec. 4.1, eq. (CT_sketches)): ray-driven Joseph forward
// projection R_l (k_fwd) and a gather-form transpose R_l^T (k_bp) that
// recomputes the forward's interpolation weights from the same FP32
// expression, so the pair is an exact transpose without atomics.  Resampling
// (block mean T_l, compensation S_r) is done by the tile-pyramid kernel
// k_prep that feeds the projector; the SAGA table refresh and the primal /
// dual proximal steps of Alg. 1 are fused into k_fwd's store (dual) and
// k_primal (primal); the smoothed-TV prox runs J FISTA iterations inside one
// launch on LDS-resident overlapped tiles (k_tv).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace imk {

namespace {

__device__ __forceinline__ bool row_stepping(int a, int na) { return 4 * a <= na || 4 * a >= 3 * na; }

constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// Left tap and right-tap weight of the fixed-point coordinate u.
__device__ __forceinline__ int tap_index(long long u) { return (int)(u >> 32); }
__device__ __forceinline__ float tap_weight(long long u) { return (float)(unsigned)(u & 0xffffffffLL) * kTwoM32; }

__global__ void k_consts(int n, int na, int nd, double ds, double s0, int lmax, RayConst* out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (lmax + 1) * na) return;
    const int l = idx / na, a = idx - l * na;
    const double th = (double)a * M_PI / (double)na;
    const double c = cos(th), s = sin(th);
    const int nl = n >> l;
    const double hl = 2.0 / nl;
    const double half = 0.5 * (nl - 1), halfd = 0.5 * (nd - 1);
    // u(i, b) = A (i - half) + B (b - halfd) + C, the column (row) coordinate
    // of ray b where it crosses row (column) i, in pixels of level l.
    double A, B, C, W;
    if (row_stepping(a, na)) {
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
    r.pad = 0;
    r.a = (float)A;
    r.b = (float)B;
    r.c = (float)C0;
    r.w = (float)W;
    r.ib = (float)(1.0 / B);
    r.r0 = r.r1 = r.r2 = 0.0f;
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

// Restricts (block mean at level l) or compensates (S_r at level 0) one
// T x T tile of x into padded row / transposed layouts for the projector.
__global__ void __launch_bounds__(256) k_prep(PrepArgs a)
{
    extern __shared__ float pyr[];
    const int tiles = a.n / a.T;
    const int ty = blockIdx.x / tiles, tx = blockIdx.x - ty * tiles;
    load_tile(pyr, a.x, a.n, a.T, ty, tx);
    build_pyramid(pyr, a.T, a.pyr_levels);
    for (int o = 0; o < a.nout; ++o) {
        const PrepOut& po = a.out[o];
        const int l = po.lvl;
        const int tl = a.T >> l, nl = a.n >> l;
        const int P = po.padded ? nl + kPad : nl;
        const int sh = po.padded ? kPadL : 0;
        const int oy = ty * tl, ox = tx * tl;
        const int off = pyr_offset(a.T, l);
        for (int q = threadIdx.x; q < tl * tl; q += blockDim.x) {
            const int i = q / tl, j = q - i * tl;
            float v = pyr[off + q];
            if (po.kind == PREP_COMP) {
                float acc = v;
                for (int c = 0; c < a.ncomp; ++c) {
                    const int lc = a.comp_lvl[c];
                    const int tc = a.T >> lc;
                    acc -= a.comp_p[c] * pyr[pyr_offset(a.T, lc) + (i >> lc) * tc + (j >> lc)];
                }
                v = acc * a.inv_p0;
            }
            po.dst[(size_t)(oy + i) * P + ox + j + sh] = v;
            if (po.dstT) po.dstT[(size_t)(ox + j) * P + oy + i + sh] = v;
        }
    }
}

// ---------------------------------------------------------- Joseph forward

// One thread per ray; each wavefront covers 64 consecutive bins of one
// angle, so the angle's constants are wavefront-uniform (scalar loads).
__global__ void __launch_bounds__(256) k_fwd(FwdArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wpa = (a.nd + 63) >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int ang = __builtin_amdgcn_readfirstlane(wave / wpa);
    if (ang >= a.na) return;
    const int b = (wave - ang * wpa) * 64 + lane;
    const bool active = b < a.nd;
    const bool rows = row_stepping(ang, a.na);
    const float fb = (float)b;
    float total = 0.0f;
    for (int q = 0; q < a.nterms; ++q) {
        const FwdTerm& t = a.term[q];
        const int nl = a.n >> t.lvl;
        const int P = nl + kPad;
        const RayConst& kc = a.consts[(size_t)t.lvl * a.na + ang];
        const float* img = rows ? t.img : t.imgT;
        const float fnl = (float)nl;
        const float tf = fmaf(fb, kc.b, kc.c);  // ~u at step 0
        // steps whose coordinate can reach [-1, nl]: a 0.01-pixel margin
        // covers the float estimate; the zero padding covers the rest
        int lo = 0, hi = nl - 1;
        if (!active) {
            lo = 1;
            hi = 0;
        } else if (kc.a != 0.0f) {
            const float s1 = (-1.01f - tf) / kc.a, s2 = (fnl + 0.01f - tf) / kc.a;
            lo = (int)fminf(fmaxf(ceilf(fminf(s1, s2)), 0.0f), fnl);
            hi = (int)fmaxf(fminf(floorf(fmaxf(s1, s2)), fnl - 1.0f), -1.0f);
        } else if (tf < -1.01f || tf > fnl + 0.01f) {
            lo = 1;
            hi = 0;
        }
        float acc = 0.0f;
        if (lo <= hi) {
            long long u = kc.cfx + (long long)b * kc.bfx + (long long)lo * kc.afx;
            const float* row = img + (size_t)lo * P + kPadL;
            int i = lo;
            // four steps per trip: all eight taps are loaded before use
            for (; i + 3 <= hi; i += 4) {
                const long long u1 = u + kc.afx, u2 = u1 + kc.afx, u3 = u2 + kc.afx;
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
                u = u3 + kc.afx;
                row += 4 * P;
            }
            for (; i <= hi; ++i) {
                const float* px = row + tap_index(u);
                const float w = tap_weight(u);
                acc = fmaf(1.0f - w, px[0], acc);
                acc = fmaf(w, px[1], acc);
                u += kc.afx;
                row += P;
            }
        }
        total = fmaf(t.coef, kc.w * acc, total);
    }
    if (!active) return;
    const size_t e = (size_t)ang * a.nd + b;
    if (a.mode == FWD_STORE) {
        a.out[e] = total;
    } else if (a.mode == FWD_ACCUM) {
        a.out[e] += total;
    } else {
        const size_t m = (size_t)a.na * a.nd;
        float avg = 0.0f;
        for (int j = 0; j < a.r; ++j) avg = fmaf(a.p[j], a.psi[(size_t)j * m + e], avg);
        const float zeta = (total - a.psi[(size_t)a.kidx * m + e]) + avg;
        a.y_new[e] = (a.y_old[e] + a.sigma * zeta - a.sigma * a.bdat[e]) * a.inv1ps;
        a.psi[(size_t)a.kidx * m + e] = total;
    }
}

// ------------------------------------------------------ gather transpose

// One thread per level-l pixel.  For every angle, the bins whose samples
// touch this pixel form a short interval; each candidate recomputes the
// forward's tap (j0, w) and keeps (1-w) if j0 is this pixel, w if it is the
// left neighbour.  No atomics: the result is deterministic.
__device__ __forceinline__ void bp_store(const BpArgs& a, int nl, int I, int J, float total)
{
    const float v = a.coef * total;
    if (!a.prolong) {
        float* o = a.out + (size_t)I * nl + J;
        *o = a.accumulate ? *o + v : v;
    } else {
        const int f = 1 << a.lvl;
        for (int di = 0; di < f; ++di) {
            float* o = a.out + (size_t)(I * f + di) * a.n + (size_t)J * f;
            for (int dj = 0; dj < f; ++dj) o[dj] = a.accumulate ? o[dj] + v : v;
        }
    }
}

// Workgroup = 16 x 16 level-l pixels x one group of angles (grid z), so the
// coarse levels, with few pixels, still fill the chip.
__global__ void __launch_bounds__(256) k_bp(BpArgs a)
{
    const int nl = a.n >> a.lvl;
    const int J = blockIdx.x * 16 + (threadIdx.x & 15);
    const int I = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (I >= nl || J >= nl) return;
    const int g = blockIdx.z;
    const int a0 = g * a.apg;
    const int a1 = min(a.na, a0 + a.apg);
    const float bmax = (float)(a.nd - 1);
    float total = 0.0f;
    const RayConst* kbase = a.consts + (size_t)a.lvl * a.na;
    for (int ang = a0; ang < a1; ++ang) {
        const RayConst& kc = kbase[ang];
        const bool rows = row_stepping(ang, a.na);
        const int s = rows ? I : J;  // step index of the samples touching this pixel
        const int q = rows ? J : I;  // interpolation index of this pixel
        // bins whose coordinate lies in (q-1, q+1): |b - bpos| < |1/B|; the
        // 1% + 0.01-bin margin covers the float estimate of bpos, the exact
        // fixed-point test below decides
        const float bpos = ((float)q - fmaf((float)s, kc.a, kc.c)) * kc.ib;
        const float R = 1.01f * fabsf(kc.ib) + 0.01f;
        const int blo = (int)fminf(fmaxf(ceilf(bpos - R), 0.0f), bmax + 1.0f);
        const int bhi = (int)fmaxf(fminf(floorf(bpos + R), bmax), -1.0f);
        float acc = 0.0f;
        if (blo <= bhi) {
            long long u = kc.cfx + (long long)s * kc.afx + (long long)blo * kc.bfx;
            const float* yr = a.y + (size_t)ang * a.nd;
            for (int b = blo; b <= bhi; ++b) {
                const int j0 = tap_index(u);
                const float w = tap_weight(u);
                const float wt = (j0 == q) ? (1.0f - w) : ((j0 == q - 1) ? w : 0.0f);
                acc = fmaf(wt, yr[b], acc);
                u += kc.bfx;
            }
        }
        total = fmaf(kc.w, acc, total);
    }
    if (a.G == 1)
        bp_store(a, nl, I, J, total);
    else
        a.part[(size_t)g * nl * nl + (size_t)I * nl + J] = total;
}

// Sums the angle-group partials in group order (deterministic) and stores.
__global__ void __launch_bounds__(256) k_bp_reduce(BpArgs a)
{
    const int nl = a.n >> a.lvl;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nl * nl) return;
    const size_t d = (size_t)nl * nl;
    float t = 0.0f;
    for (int g = 0; g < a.G; ++g) t += a.part[g * d + q];
    bp_store(a, nl, q / nl, q % nl, t);
}

// ------------------------------------------------------------ primal step

// Forms phi_new = K_k^T y at full resolution from the raw backprojections,
// the SAGA estimate xi with the old tables, v = x - tau xi, and writes
// prox_scale * v; then refreshes table k.  One workgroup per T x T tile
// (T a multiple of every level's block, so coarse cells never straddle).
__global__ void __launch_bounds__(256) k_primal(PrimalArgs a)
{
    extern __shared__ float pyr[];
    const int tiles = a.n / a.T;
    const int ty = blockIdx.x / tiles, tx = blockIdx.x - ty * tiles;
    const bool paper_full = (a.kidx == 0 && a.full_mode == IMASK_FULL_PAPER && a.r > 1);
    if (paper_full) {
        load_tile(pyr, a.craw[0], a.n, a.T, ty, tx);
        build_pyramid(pyr, a.T, a.pyr_levels);
    }
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
        for (int c = 0; c < a.r; ++c) {
            float ph;
            if (c == 0) {
                ph = a.phi[a.phi_off[0] + pix];
            } else {
                const int l = a.lvl[c];
                const int nl = a.n >> l;
                ph = a.phi[a.phi_off[c] + (size_t)(i >> l) * nl + (j >> l)];
            }
            avg = fmaf(a.p[c], ph, avg);
            if (c == a.kidx) own = ph;
        }
        const float xi = (g - own) + avg;
        const float v = a.x_old[pix] - a.tau * xi;
        a.x_out[pix] = v * a.prox_scale;
        if (a.kidx == 0) a.phi[a.phi_off[0] + pix] = g;
    }
    if (a.kidx > 0) {
        __syncthreads();  // every old phi_k value of this tile has been read
        const int l = a.lvl[a.kidx];
        const int nl = a.n >> l, tl = a.T >> l;
        const float s = 1.0f / (float)(1 << (2 * l));
        for (int qq = threadIdx.x; qq < tl * tl; qq += blockDim.x) {
            const int ci = ty * tl + qq / tl, cj = tx * tl + (qq % tl);
            const size_t c = (size_t)ci * nl + cj;
            a.phi[a.phi_off[a.kidx] + c] = a.craw[a.kidx][c] * s;
        }
    }
}

// ------------------------------------------------------------ smoothed TV

// J FISTA iterations of the prox of tau*(w TV_eps + lam/2 |.|^2) on one
// 32 x 32 output tile; the workgroup holds the tile plus a J-pixel halo in
// LDS and shrinks the valid region by one pixel per iteration, so the whole
// inner solve reads v and u0 once and writes the result once.
constexpr int kTvTile = 32;

__global__ void __launch_bounds__(256) k_tv(TvArgs a)
{
    extern __shared__ float sm[];
    const int H = a.J;
    const int R = kTvTile + 2 * H;
    float* vs = sm;
    float* up = vs + R * R;
    float* ys = up + R * R;
    float* q1 = ys + R * R;
    float* q2 = q1 + R * R;
    const int tiles = (a.n + kTvTile - 1) / kTvTile;
    const int ty = blockIdx.x / tiles, tx = blockIdx.x - ty * tiles;
    const int gi0 = ty * kTvTile - H, gj0 = tx * kTvTile - H;
    const int n = a.n;
    for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
        const int li = q / R, lj = q - li * R;
        const int gi = gi0 + li, gj = gj0 + lj;
        float v = 0.f, u = 0.f;
        if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
            v = a.v[(size_t)gi * n + gj];
            u = a.u0[(size_t)gi * n + gj];
        }
        vs[q] = v;
        up[q] = u;
        ys[q] = u;
    }
    __syncthreads();
    for (int t = 0; t < a.J; ++t) {
        // q = grad y / sqrt(|grad y|^2 + eps^2) on [t, R-2-t]^2
        const int lo = t, hiq = R - 2 - t;
        const int wq = hiq - lo + 1;
        for (int q = threadIdx.x; q < wq * wq; q += blockDim.x) {
            const int li = lo + q / wq, lj = lo + q % wq;
            const int gi = gi0 + li, gj = gj0 + lj;
            if (gi < 0 || gi >= n || gj < 0 || gj >= n) continue;
            const int c = li * R + lj;
            const float yc = ys[c];
            const float d1 = (gi < n - 1) ? ys[c + R] - yc : 0.0f;
            const float d2 = (gj < n - 1) ? ys[c + 1] - yc : 0.0f;
            const float inv = 1.0f / sqrtf(d1 * d1 + d2 * d2 + a.eps * a.eps);
            q1[c] = d1 * inv;
            q2[c] = d2 * inv;
        }
        __syncthreads();
        const int lo2 = t + 1, hi2 = R - 2 - t;
        const int w2 = hi2 - lo2 + 1;
        const float beta = a.beta[t];
        for (int q = threadIdx.x; q < w2 * w2; q += blockDim.x) {
            const int li = lo2 + q / w2, lj = lo2 + q % w2;
            const int gi = gi0 + li, gj = gj0 + lj;
            if (gi < 0 || gi >= n || gj < 0 || gj >= n) continue;
            const int c = li * R + lj;
            float div = -q1[c] - q2[c];  // grad^T q
            if (gi >= 1) div += q1[c - R];
            if (gj >= 1) div += q2[c - 1];
            const float yc = ys[c];
            const float gh = (yc - vs[c]) + a.tau_w * div + a.tau_lam * yc;
            const float un = yc - a.invL * gh;
            ys[c] = un + beta * (un - up[c]);
            up[c] = un;
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < kTvTile * kTvTile; q += blockDim.x) {
        const int li = H + q / kTvTile, lj = H + q % kTvTile;
        const int gi = gi0 + li, gj = gj0 + lj;
        if (gi < n && gj < n) a.out[(size_t)gi * n + gj] = up[li * R + lj];
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

}  // namespace

// ----------------------------------------------------------------- launchers

int tile_side(int n, int lmax)
{
    int T = 16 < n ? 16 : n;
    while (T < (1 << lmax)) T <<= 1;
    return T;
}

hipError_t launch_consts(const imask_geometry& g, const Layout& L, float* work, hipStream_t s)
{
    const double ds = g.det_spacing > 0 ? g.det_spacing : 2.0 / g.n;
    const int count = (L.lmax + 1) * g.n_angles;
    hipLaunchKernelGGL(k_consts, dim3((count + 255) / 256), dim3(256), 0, s, g.n, g.n_angles, g.n_det, ds,
                       g.det_offset, L.lmax, (RayConst*)(work + L.consts));
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
    const int tiles = a.n / a.T;
    hipLaunchKernelGGL(k_prep, dim3(tiles * tiles), dim3(256), pyramid_bytes(a.T, a.pyr_levels), s, a);
    return hipGetLastError();
}

hipError_t launch_fwd(const FwdArgs& a, hipStream_t s)
{
    const int wpa = (a.nd + 63) / 64;
    const long waves = (long)wpa * a.na;
    hipLaunchKernelGGL(k_fwd, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bp(const BpArgs& a0, hipStream_t s)
{
    BpArgs a = a0;
    const int nl = a.n >> a.lvl;
    const int t = (nl + 15) / 16;
    // enough angle groups for ~1024 workgroups, within the 4 N^2 partial buffer
    const int gmax = std::min(a.na, 4 << (2 * a.lvl));
    int G = std::max(1, std::min(gmax, (1024 + t * t - 1) / (t * t)));
    a.apg = (a.na + G - 1) / G;
    a.G = (a.na + a.apg - 1) / a.apg;
    hipLaunchKernelGGL(k_bp, dim3(t, t, a.G), dim3(256), 0, s, a);
    if (a.G > 1) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_bp_reduce, dim3((nl * nl + 255) / 256), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_primal(const PrimalArgs& a, hipStream_t s)
{
    const int tiles = a.n / a.T;
    const bool paper_full = (a.kidx == 0 && a.full_mode == IMASK_FULL_PAPER && a.r > 1);
    const size_t sh = paper_full ? pyramid_bytes(a.T, a.pyr_levels) : 0;
    hipLaunchKernelGGL(k_primal, dim3(tiles * tiles), dim3(256), sh, s, a);
    return hipGetLastError();
}

hipError_t launch_tv(const TvArgs& a, hipStream_t s)
{
    const int R = kTvTile + 2 * a.J;
    const size_t sh = (size_t)5 * R * R * sizeof(float);
    const int tiles = (a.n + kTvTile - 1) / kTvTile;
    hipLaunchKernelGGL(k_tv, dim3(tiles * tiles), dim3(256), sh, s, a);
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
