// Per-pixel compositing (forward and backward).
//
// Work decomposition: one wavefront (64 lanes) owns one screen tile of
// TW x TH pixels, cut into TW * TH / 64 pixel slots (slot_layout in
// binning.h: 8 x 8 blocks, or full-width row bands); lane l holds one pixel
// of every slot, and a slot whose culling bit is clear, or whose pixels have
// all stopped, is skipped by the whole wave.  Waves of a workgroup are
// independent: each pulls tile ids
// from one of kQueues atomic queues (persistent grid; the queues interleave
// the heavy-first work order, and splitting the head keeps one memory
// address from serialising every take), stages 64 raster records at a
// time in its own LDS slice and reads them back as broadcasts, and leaves the
// tile as soon as a ballot shows that no lane has a live pixel (early ray
// termination).  No workgroup barrier is ever taken.
//
// Per fragment (Sec. 4.2, eq. 16): with delta the pixel-centre offset from the
// projected centre, n = G delta is the quad-plane offset times den and
// den = k0 + g . delta is proportional to x^T Sigma^-1 mu (> 0 iff tau > 0),
// so |zeta|^2 = q / den^2 with q = |n|^2 and
//     D = (c^-2 + |zeta|^-2)^-1 = q / (den^2 + q / c^2),
// a form without the cancellation of c^2 - (x^T Sigma^-1 mu)^2 / x^T Sigma^-1 x.
// omega = o exp(-D/2) (eq. 2); a Gaussian contributes iff den > 0 and
// omega >= p_min; alpha = min(omega, alpha_max); compositing (eq. 1) stops
// before a Gaussian that would take T below t_eps.
//
// The loops read each record in a test form made when it is staged: with
// K = log2(o / p_min) and s^2 = log2(e) / (2 K), H = s G and j = ic2 / s^2,
// qs = |H delta|^2 = s^2 q and t = den^2 + qs j = den^2 + q / c^2, so the
// exponent D log2(e) / 2 equals K qs / t and omega >= p_min reads qs <= t.
#include <hip/hip_fp16.h>

#include <algorithm>

#include "internal.h"

#pragma clang fp contract(off)

namespace rgs {
namespace {

// Test form of a raster record for one tile (four float4 in LDS).  Positions
// are taken relative to the corner of the 32 x 32 pixel block that holds the
// tile: a tile of any supported shape lies inside one such block, so every
// pixel gets the same arithmetic whatever the tile shape, and offsets from
// the corner are small exact integers.
//   [0] cx, cy, K, rows   projected centre minus the block corner;
//                          K = log2(o / p_min); covered rows or slot bits
//   [1] H00 H01 H10 H11   H = s G
//   [2] gx, gy, k0, j     j = ic2 / s^2
//   [3] log2o, r, g, b
struct TRec {
    float cx, cy, K, H00, H01, H10, H11, gx, gy, k0, j, log2o, r, g, b;
    uint32_t rows;  // first | last << 16 covered pixel row, or the instance's slot bits
};

struct Frag {
    float dx, dy, n0, n1, den, q, t, rt, w;
};

__device__ __forceinline__ TRec load_trec(const float4 *p)
{
    const float4 a = p[0], b = p[1], c = p[2], d = p[3];
    return TRec{a.x, a.y, a.z, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w, __float_as_uint(a.w)};
}

constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
constexpr float kTwoLn2 = 1.38629436111989061f;     // 2 / log2(e)

// The per-fragment instruction sequence shared by the forward and the
// backward kernel (explicit fma, no contraction), so both take identical
// decisions.  (pxr, pyr) is the pixel centre relative to the block corner;
// a NaN pyr (a pixel that is done) fails every comparison.
// frag_test decides whether the Gaussian contributes: den > 0 (tau > 0) and
// omega >= p_min, i.e. qs <= t, without a reciprocal or exponential.
// frag_omega then finishes omega = o 2^(-K qs / t) for accepted fragments.
__device__ __forceinline__ bool frag_test(const TRec &R, float pxr, float pyr, Frag &f)
{
    f.dx = pxr - R.cx;
    f.dy = pyr - R.cy;
    f.n0 = __builtin_fmaf(R.H01, f.dy, R.H00 * f.dx);
    f.n1 = __builtin_fmaf(R.H11, f.dy, R.H10 * f.dx);
    f.den = __builtin_fmaf(R.gy, f.dy, __builtin_fmaf(R.gx, f.dx, R.k0));
    f.q = __builtin_fmaf(f.n1, f.n1, f.n0 * f.n0);
    f.t = __builtin_fmaf(f.q, R.j, f.den * f.den);
    return (f.den > 0.0f) & (f.q <= f.t);
}

__device__ __forceinline__ void frag_omega(const TRec &R, Frag &f)
{
    f.rt = __builtin_amdgcn_rcpf(f.t);
    f.w = __builtin_amdgcn_exp2f(__builtin_fmaf(R.K * f.q, -f.rt, R.log2o));
}

// Rows of the tile covered by a record, relative to the tile's first row, as
// wave-uniform (scalar) values: where the tile's slots carry no bits, a slot
// whose rows lie outside [r0, r1] is skipped by the whole wave.
struct RowSpan {
    int r0, r1;
};

__device__ __forceinline__ RowSpan row_span(uint32_t rows_word, int tile_row0)
{
    const uint32_t rows = __builtin_amdgcn_readfirstlane(rows_word);
    return RowSpan{(int)(rows & 0xffffu) - tile_row0, (int)(rows >> 16) - tile_row0};
}

__device__ __forceinline__ void lds_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int find_view(const DevView *views, int n_views, int tile)
{
    int v = 0;
    while (v + 1 < n_views && views[v + 1].tile_base <= tile) ++v;
    return v;
}

struct BlendParams {
    float log2_pmin, alpha_max, t_eps, bg0, bg1, bg2;
    int n_views, total_tiles;
    uint32_t n_records;
    unsigned long long *item_clock;  // per work-order slot: wall clock at the item's end (may be null)
};

// Raw record (four float4) of instance value `inst` (id | slot bits),
// fetched ahead of its conversion.  An id outside the record array (never
// produced by the binning) gets a placeholder that cannot reach p_min.  When
// the tile's slots carry bits the covered-rows word is not needed, and the
// instance's slot bits take its place.
__device__ __forceinline__ void fetch_record(float4 (&r)[4], const float4 *__restrict__ records, uint32_t inst,
                                             uint32_t n_records, bool bands_in_rows)
{
    const uint32_t id = inst & kIdMask;
    if (id < n_records) {
        const float4 *src = records + (size_t)id * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] = src[c];
    } else {
        r[0] = make_float4(0.f, 0.f, 0.f, __uint_as_float(1u));  // rows [1, 0]: empty
        r[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        r[2] = make_float4(0.f, 0.f, -1.f, 0.f);
        r[3] = make_float4(-126.f, 0.f, 0.f, 0.f);
    }
    if (bands_in_rows) r[0].w = __uint_as_float(inst >> kIdBits);
}

// Writes the test form of raw record r for the tile whose block corner is
// (x0, y0).  A record with K <= 0 in FP32 (which includes the
// placeholder) cannot reach p_min and gets den = -1 everywhere.
__device__ __forceinline__ void put_test_form(float4 *dst, const float4 (&r)[4], float x0, float y0,
                                              float log2_pmin)
{
    const uint32_t lo_bits = __float_as_uint(r[0].z);
    const float2 lo = __half22float2(*reinterpret_cast<const __half2 *>(&lo_bits));
    const float K = r[3].x - log2_pmin;
    const float rows = r[0].w;
    if (K > 0.0f) {
        const float s = __builtin_amdgcn_sqrtf(kHalfLog2e * __builtin_amdgcn_rcpf(K));
        dst[0] = make_float4((r[0].x - x0) + lo.x, (r[0].y - y0) + lo.y, K, rows);
        dst[1] = make_float4(s * r[1].x, s * r[1].y, s * r[1].z, s * r[1].w);
        dst[2] = make_float4(r[2].x, r[2].y, r[2].z, (K * kTwoLn2) * r[2].w);
    } else {
        dst[0] = make_float4(0.f, 0.f, 1.f, rows);
        dst[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        dst[2] = make_float4(0.f, 0.f, -1.f, 0.f);
    }
    dst[3] = r[3];
}

// Record model of the forward kernel: how a raw record is fetched, staged
// in LDS for one tile, read back, and tested per fragment.  PlainModel is the
// record above (with or without the approximate MIP of eq. 17, which only
// changes the record's values); ExactMipModel evaluates the exact MIP weight.
struct PlainModel {
    static constexpr int kRaw = 4, kStaged = 4;
    using Rec = TRec;
    using F = Frag;
    __device__ static float pixel_aux(const DevView &, int, int) { return 0.0f; }
    __device__ static void fetch(float4 (&r)[kRaw], const float4 *__restrict__ records, uint32_t inst,
                                 uint32_t n_records, bool bands_in_rows)
    {
        fetch_record(r, records, inst, n_records, bands_in_rows);
    }
    // the same in two steps: loads with no branch (the id clamped into the
    // record array, n_records >= 1), then what fetch decides by branching
    __device__ static void load_raw(float4 (&r)[kRaw], const float4 *__restrict__ records, uint32_t inst,
                                    uint32_t n_records)
    {
        const float4 *src = records + (size_t)min(inst & kIdMask, n_records - 1u) * kRaw;
#pragma unroll
        for (int c = 0; c < kRaw; ++c) r[c] = src[c];
    }
    __device__ static void settle(float4 (&r)[kRaw], uint32_t inst, uint32_t n_records, bool bands_in_rows)
    {
        if ((inst & kIdMask) >= n_records) {
            r[0] = make_float4(0.f, 0.f, 0.f, __uint_as_float(1u));
            r[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            r[2] = make_float4(0.f, 0.f, -1.f, 0.f);
            r[3] = make_float4(-126.f, 0.f, 0.f, 0.f);
        }
        if (bands_in_rows) r[0].w = __uint_as_float(inst >> kIdBits);
    }
    __device__ static void stage(float4 *dst, const float4 (&r)[kRaw], float x0, float y0, float log2_pmin)
    {
        put_test_form(dst, r, x0, y0, log2_pmin);
    }
    __device__ static Rec load(const float4 *p) { return load_trec(p); }
    __device__ static bool test(const Rec &R, float pxr, float pyr, float, float, F &f)
    {
        return frag_test(R, pxr, pyr, f);
    }
    __device__ static float omega(const Rec &R, F &f)
    {
        frag_omega(R, f);
        return f.w;
    }
};

// Exact MIP (mip = 2).  The record (seven float4, written by the preprocess
// kernel) describes the Gaussian in its own axes, scaled so that the largest
// variance is 1 (lam = s_max^2):
//   [0] u_hi, v_hi, lo, rows      projected centre and covered rows, as above
//   [1] P0 (3), e                 P0 = R_p^T e_x / f_x;  e = sigma^2 mu_z^2 / lam
//   [2] P1 (3), log2o             P1 = R_p^T e_y / f_y;  log2o = log2 o + log2 sqrt(prod s'^2)
//   [3] Q0 (3), r                 Q0 = R_p^T (0, 1, -v0) mu_z / (f_x sqrt(lam))
//   [4] Q1 (3), g                 Q1 = R_p^T (-1, 0, u0) mu_z / (f_y sqrt(lam))
//   [5] rho (3), b                rho = R_p^T mu / mu_z
//   [6] s'^2 (3), 0               s'^2 = s^2 / lam
// For a pixel offset delta from the projected centre, the ray xbar = (u, v, 1)
// has r = R_p^T xbar = rho + P0 dx + P1 dy, and w = Q0 dx + Q1 dy is
// R_p^T (mu x xbar) (scaled), linear in delta with no cancellation.  With
// A = sum rho_k r_k / s'_k^2 and B = sum r_k^2 / s'_k^2, the widening of
// this ray is a = e |xbar|^-1 (A / B)^2 (sigma_x^2 tau(x)^2 over lam), the
// widened variances S_k = s'_k^2 + a, and with
//   den = sum_k r_k^2 prod_{j != k} S_j,   num = sum_k S_k w_k^2,
// D_ray(x; mu, Sigma^_x) = num / den (the cross-product form of
// c^2 - (x.mu)^2 / x.x in the widened metric), the modulation is
// m^2 = prod s'^2 B / den, and the peak of the widened density lies in front
// iff sum_k rho_k r_k prod_{j != k} S_j > 0.  Every sum has positive terms
// except A, which only sets the widening.  omega = 2^L with
// L = log2o + log2(B / den) / 2 - num log2(e) / (2 den).
struct XRec {
    float cx, cy, e, P0x, P0y, P0z, P1x, P1y, P1z, Q0x, Q0y, Q0z, Q1x, Q1y, Q1z;
    float rx, ry, rz, log2o, ix_, iy_, iz_, r, isx, isy, isz, g, s0, s1, s2, b;
    uint32_t rows;
};

// Per-fragment values of the exact MIP weight (the backward kernel uses
// them all; the forward only L).
struct XFrag {
    float dx, dy, r0, r1, r2, w0, w1, w2, q0, q1, q2, rB, t, S0, S1, S2, p12, p02, p01, den, num, rd, L;
};

struct ExactMipModel {
    static constexpr int kRaw = 7, kStaged = 8;
    using Rec = XRec;
    using F = XFrag;
    // 1 / |xbar| of the pixel-centre ray (the footprint's cos(theta))
    __device__ static float pixel_aux(const DevView &V, int px, int py)
    {
        const float u = ((float)px + 0.5f - (float)V.cx) * (float)(1.0 / V.fx);
        const float v = ((float)py + 0.5f - (float)V.cy) * (float)(1.0 / V.fy);
        return __builtin_amdgcn_rsqf(__builtin_fmaf(v, v, __builtin_fmaf(u, u, 1.0f)));
    }
    __device__ static void fetch(float4 (&r)[kRaw], const float4 *__restrict__ records, uint32_t inst,
                                 uint32_t n_records, bool bands_in_rows)
    {
        const uint32_t id = inst & kIdMask;
        if (id < n_records) {
            const float4 *src = records + (size_t)id * kRaw;
#pragma unroll
            for (int c = 0; c < kRaw; ++c) r[c] = src[c];
        } else {
            // rows [1, 0]: empty; a ray in front with omega = 2^-126
            r[0] = make_float4(0.f, 0.f, 0.f, __uint_as_float(1u));
            r[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            r[2] = make_float4(0.f, 0.f, 0.f, -126.f);
            r[3] = make_float4(0.f, 0.f, 0.f, 0.f);
            r[4] = make_float4(0.f, 0.f, 0.f, 0.f);
            r[5] = make_float4(0.f, 0.f, 1.f, 0.f);
            r[6] = make_float4(1.f, 1.f, 1.f, 0.f);
        }
        if (bands_in_rows) r[0].w = __uint_as_float(inst >> kIdBits);
    }
    __device__ static void load_raw(float4 (&r)[kRaw], const float4 *__restrict__ records, uint32_t inst,
                                    uint32_t n_records)
    {
        const float4 *src = records + (size_t)min(inst & kIdMask, n_records - 1u) * kRaw;
#pragma unroll
        for (int c = 0; c < kRaw; ++c) r[c] = src[c];
    }
    __device__ static void settle(float4 (&r)[kRaw], uint32_t inst, uint32_t n_records, bool bands_in_rows)
    {
        if ((inst & kIdMask) >= n_records) {
            r[0] = make_float4(0.f, 0.f, 0.f, __uint_as_float(1u));
            r[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            r[2] = make_float4(0.f, 0.f, 0.f, -126.f);
            r[3] = make_float4(0.f, 0.f, 0.f, 0.f);
            r[4] = make_float4(0.f, 0.f, 0.f, 0.f);
            r[5] = make_float4(0.f, 0.f, 1.f, 0.f);
            r[6] = make_float4(1.f, 1.f, 1.f, 0.f);
        }
        if (bands_in_rows) r[0].w = __uint_as_float(inst >> kIdBits);
    }
    // staged: [0] cx cy e rows [1] P0 P1x [2] P1yz Q0xy [3] Q0z Q1 [4] rho log2o
    //         [5] rho/s'^2 r [6] 1/s'^2 g [7] s'^2 b
    __device__ static void stage(float4 *dst, const float4 (&r)[kRaw], float x0, float y0, float)
    {
        const uint32_t lo_bits = __float_as_uint(r[0].z);
        const float2 lo = __half22float2(*reinterpret_cast<const __half2 *>(&lo_bits));
        const float isx = 1.0f / r[6].x, isy = 1.0f / r[6].y, isz = 1.0f / r[6].z;
        dst[0] = make_float4((r[0].x - x0) + lo.x, (r[0].y - y0) + lo.y, r[1].w, r[0].w);
        dst[1] = make_float4(r[1].x, r[1].y, r[1].z, r[2].x);
        dst[2] = make_float4(r[2].y, r[2].z, r[3].x, r[3].y);
        dst[3] = make_float4(r[3].z, r[4].x, r[4].y, r[4].z);
        dst[4] = make_float4(r[5].x, r[5].y, r[5].z, r[2].w);
        dst[5] = make_float4(r[5].x * isx, r[5].y * isy, r[5].z * isz, r[3].w);
        dst[6] = make_float4(isx, isy, isz, r[4].w);
        dst[7] = make_float4(r[6].x, r[6].y, r[6].z, r[5].w);
    }
    __device__ static Rec load(const float4 *p)
    {
        const float4 a = p[0], b = p[1], c = p[2], d = p[3], e = p[4], f = p[5], g = p[6], h = p[7];
        return XRec{a.x, a.y, a.z, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w,
                    e.x, e.y, e.z, e.w, f.x, f.y, f.z, f.w, g.x, g.y, g.z, g.w, h.x, h.y, h.z, h.w,
                    __float_as_uint(a.w)};
    }
    __device__ static bool test(const Rec &R, float pxr, float pyr, float inv_norm, float log2_pmin, F &f)
    {
        const float dx = pxr - R.cx, dy = pyr - R.cy;
        const float r0 = __builtin_fmaf(R.P1x, dy, __builtin_fmaf(R.P0x, dx, R.rx));
        const float r1 = __builtin_fmaf(R.P1y, dy, __builtin_fmaf(R.P0y, dx, R.ry));
        const float r2 = __builtin_fmaf(R.P1z, dy, __builtin_fmaf(R.P0z, dx, R.rz));
        const float w0 = __builtin_fmaf(R.Q1x, dy, R.Q0x * dx);
        const float w1 = __builtin_fmaf(R.Q1y, dy, R.Q0y * dx);
        const float w2 = __builtin_fmaf(R.Q1z, dy, R.Q0z * dx);
        const float A = __builtin_fmaf(R.iz_, r2, __builtin_fmaf(R.iy_, r1, R.ix_ * r0));
        const float q0 = r0 * r0, q1 = r1 * r1, q2 = r2 * r2;
        const float B = __builtin_fmaf(R.isz, q2, __builtin_fmaf(R.isy, q1, R.isx * q0));
        const float rB = __builtin_amdgcn_rcpf(B);
        const float t = A * rB;
        const float a = (R.e * inv_norm) * (t * t);
        const float S0 = R.s0 + a, S1 = R.s1 + a, S2 = R.s2 + a;
        const float p12 = S1 * S2, p02 = S0 * S2, p01 = S0 * S1;
        const float den = __builtin_fmaf(q2, p01, __builtin_fmaf(q1, p02, q0 * p12));
        const float num = __builtin_fmaf(S2, w2 * w2, __builtin_fmaf(S1, w1 * w1, S0 * (w0 * w0)));
        const float th = __builtin_fmaf(R.rz * r2, p01, __builtin_fmaf(R.ry * r1, p02, (R.rx * r0) * p12));
        const float rd = __builtin_amdgcn_rcpf(den);
        f.L = __builtin_fmaf(-kHalfLog2e * num, rd, __builtin_fmaf(0.5f, __builtin_amdgcn_logf(B * rd), R.log2o));
        f.dx = dx;
        f.dy = dy;
        f.r0 = r0;
        f.r1 = r1;
        f.r2 = r2;
        f.w0 = w0;
        f.w1 = w1;
        f.w2 = w2;
        f.q0 = q0;
        f.q1 = q1;
        f.q2 = q2;
        f.rB = rB;
        f.t = t;
        f.S0 = S0;
        f.S1 = S1;
        f.S2 = S2;
        f.p12 = p12;
        f.p02 = p02;
        f.p01 = p01;
        f.den = den;
        f.num = num;
        f.rd = rd;
        return (th > 0.0f) & (f.L >= log2_pmin);
    }
    __device__ static float omega(const Rec &, F &f) { return __builtin_amdgcn_exp2f(f.L); }
};

// Whether slot k of the tile may hold a fragment of the record: its culling
// bit when the tile's slots carry bits (`bands` is then the record's rows
// word with the instance's bits in it), else the record's covered rows
// against the slot's rows (the slots are then full-width row bands).
template <int TW, int TH>
__device__ __forceinline__ bool band_open(uint32_t bands, const RowSpan &span, int k)
{
    constexpr SlotLayout SL = slot_layout(TW, TH);
    if (SL.bits) return (bands >> k) & 1u;
    return !(span.r1 < k * SL.rh || span.r0 >= (k + 1) * SL.rh);
}

// Pixel of a lane in slot k, relative to the tile's first pixel.
template <int TW, int TH>
__device__ __forceinline__ int slot_x(int lane, int k)
{
    constexpr SlotLayout SL = slot_layout(TW, TH);
    return SL.cw * (k % SL.bx) + lane % SL.cw;
}

template <int TW, int TH>
__device__ __forceinline__ int slot_y(int lane, int k)
{
    constexpr SlotLayout SL = slot_layout(TW, TH);
    return SL.rh * (k / SL.bx) + lane / SL.cw;
}

template <int TW, int TH, class M>
__global__ __launch_bounds__(256) void k_blend(const uint2 *__restrict__ ranges,
                                               const uint32_t *__restrict__ work_order,
                                               const uint32_t *__restrict__ n_items_p,
                                               const uint32_t *__restrict__ inst_ids,
                                               const float4 *__restrict__ records, const DevView *__restrict__ views,
                                               BlendParams P, unsigned int *__restrict__ queue)
{
    constexpr int PPL = slot_layout(TW, TH).slots;
    static_assert(64 % TW == 0 && PPL * 64 == TW * TH, "tile shape");
    __shared__ float4 s_rec[4][64][M::kStaged];
    const uint32_t amax_bits = __float_as_uint(P.alpha_max);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nq = min((int)gridDim.x, kQueues), q = (int)blockIdx.x % nq;
    unsigned int *const head = queue + q * kQueueStride;
    const int64_t n_items = *n_items_p;
    for (;;) {
        const int64_t slot = q + (int64_t)nq * wave_fetch_add(head, 1u);
        if (slot >= n_items) break;
        const uint32_t item = work_order[slot];
        const int tile = (int)(item >> 2);
        // pixel slots [k_lo, k_hi) of the lanes: all, or one half of the rows
        const int part = (int)(item & 3u);
        const int k_lo = part == 2 ? PPL / 2 : 0, k_hi = part == 1 ? PPL / 2 : PPL;
        const DevView &V = views[find_view(views, P.n_views, tile)];
        const int local = tile - V.tile_base;
        const int tx = local % V.tiles_x, ty = local / V.tiles_x;
        const int ox = (tx * TW) & ~31, oy = (ty * TH) & ~31;
        const float x0 = (float)ox, y0 = (float)oy;
        // pixel centres relative to the block corner; NaN marks a pixel that
        // is outside the image, outside the work item, or done
        const uint2 rg = ranges[tile];
        float T[PPL], C0[PPL], C1[PPL], C2[PPL], pxr[PPL], pyr[PPL], aux[PPL];
        int last[PPL];
        // pixel slots (64 pixels each) that hold a live pixel: a slot
        // whose pixels have all stopped is skipped by the whole wave
        uint32_t live = 0u;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int px = tx * TW + slot_x<TW, TH>(lane, k), py = ty * TH + slot_y<TW, TH>(lane, k);
            const bool on = k >= k_lo && k < k_hi && px < V.width && py < V.height;
            pxr[k] = (float)(px - ox) + 0.5f;
            pyr[k] = on ? (float)(py - oy) + 0.5f : __builtin_nanf("");
            aux[k] = M::pixel_aux(V, px, py);
            T[k] = 1.0f;
            C0[k] = C1[k] = C2[k] = 0.0f;
            // entries consumed: the whole list unless compositing stops
            last[k] = (int)(rg.y - rg.x);
            if (__ballot(on) != 0) live |= 1u << k;
        }
        bool wave_live = live != 0u;
        // Batch 0 goes straight to LDS.  While batch b is composited, the
        // raw records of batch b + 1 and the ids of batch b + 2 are in
        // flight: their loads carry no branch (indices clamped into the
        // list, ids into the record array), so the wait for them falls after
        // the batch, where they are converted and staged.
        if (rg.x < rg.y) {
        if (rg.x + lane < rg.y) {
            const uint32_t inst = inst_ids[rg.x + lane];
            float4 r[M::kRaw];
            M::fetch(r, records, inst, P.n_records, PPL <= 4);
            M::stage(s_rec[wave][lane], r, x0, y0, P.log2_pmin);
        }
        uint32_t nid = inst_ids[min(rg.x + 64 + lane, rg.y - 1u)];
        for (uint32_t base = rg.x; base < rg.y && wave_live; base += 64) {
            const uint32_t nb = min(64u, rg.y - base);
            const bool have_next = base + 64 + lane < rg.y;
            const uint32_t cid = nid;
            float4 raw[M::kRaw];
            M::load_raw(raw, records, cid, P.n_records);
            nid = inst_ids[min(base + 128 + lane, rg.y - 1u)];
            lds_wave_sync();
            for (uint32_t j = 0; j < nb; ++j) {
                const typename M::Rec R = M::load(s_rec[wave][j]);
                const RowSpan span = row_span(R.rows, ty * TH);
                const uint32_t bands = __builtin_amdgcn_readfirstlane(R.rows);
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    if (!((live >> k) & 1u) || !band_open<TW, TH>(bands, span, k)) continue;
                    // every lane evaluates the test; results are kept by selection
                    // (the values are those of a branch per lane, bit for bit)
                    typename M::F f;
                    const bool hit = M::test(R, pxr[k], pyr[k], aux[k], P.log2_pmin, f);
                    if (__ballot(hit) == 0) continue;
                    // omega >= 0 and alpha_max > 0: the float minimum is the
                    // minimum of the bit patterns.  A lane without a hit takes
                    // alpha = 0, which leaves T and C as they are; since T >=
                    // t_eps holds for every pixel (a stopped one keeps the T
                    // from before its stop), only a hit can stop a pixel.
                    const float w = M::omega(R, f);
                    const float a = hit ? __uint_as_float(min(__float_as_uint(w), amax_bits)) : 0.0f;
                    const float ta = T[k] * a;
                    const float Tn = T[k] - ta;
                    const bool stop = Tn < P.t_eps;
                    const float wt = stop ? 0.0f : ta;
                    C0[k] = __builtin_fmaf(wt, R.r, C0[k]);
                    C1[k] = __builtin_fmaf(wt, R.g, C1[k]);
                    C2[k] = __builtin_fmaf(wt, R.b, C2[k]);
                    T[k] = stop ? T[k] : Tn;
                    if (__ballot(stop) != 0) {
                        // some pixel of the slot stops before this entry: it has
                        // consumed the entries before it, and it is done (a NaN
                        // row offset fails every later test)
                        last[k] = stop ? (int)(base - rg.x + j) : last[k];
                        pyr[k] = stop ? __builtin_nanf("") : pyr[k];
                        if (__ballot(pyr[k] == pyr[k]) == 0) live &= ~(1u << k);
                    }
                }
                // leave the tile once no pixel is live
                if (live == 0u) {
                    wave_live = false;
                    break;
                }
            }
            lds_wave_sync();
            if (have_next) {
                M::settle(raw, cid, P.n_records, PPL <= 4);
                M::stage(s_rec[wave][lane], raw, x0, y0, P.log2_pmin);
            }
        }
        }
        const size_t plane = (size_t)V.width * V.height;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int px = tx * TW + slot_x<TW, TH>(lane, k), py = ty * TH + slot_y<TW, TH>(lane, k);
            if (k >= k_lo && k < k_hi && px < V.width && py < V.height) {
                const size_t p = (size_t)py * V.width + px;
                V.rgb[p] = C0[k] + T[k] * P.bg0;
                V.rgb[plane + p] = C1[k] + T[k] * P.bg1;
                V.rgb[2 * plane + p] = C2[k] + T[k] * P.bg2;
                V.final_T[p] = T[k];
                V.n_contrib[p] = last[k];
            }
        }
        // completion clock of the item (every lane stores the same value)
        if (P.item_clock != nullptr) P.item_clock[slot] = wall_clock64();
    }
}

// Sums of 16 per-lane values over the wave by transposing while reducing:
// at each step a lane keeps one half of its values and takes its partner's
// copy of them, so 16 sums take 8 + 4 + 2 + 1 exchanges plus two for the last
// value instead of 16 * 6.  The exchanges between the halves and quarters of
// the wave are lane swaps (v_permlane32_swap / v_permlane16_swap: the two
// halves of a pair of registers trade places, so the sum of the pair holds
// one value's sum in each half); those inside 16-lane rows are DPP operands
// (row_ror:8, row_half_mirror, quad_perm).  On return, lane l holds the sum of
// value index ((l >> 5) & 1) * 8 + ((l >> 4) & 1) * 4 + ((l >> 3) & 1) * 2 +
// ((l >> 2) & 1) (the same in the four lanes l & ~3 .. l | 3).
__device__ __forceinline__ float lane_swap_sum32(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float lane_swap_sum16(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// x from the lane chosen by a DPP control word (a permutation inside each row)
template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

constexpr int kDppRowRor8 = 0x128;        // lane i of a row takes lane (i + 8) mod 16
constexpr int kDppRowHalfMirror = 0x141;  // lane i of an 8-lane group takes lane 7 - i
constexpr int kDppQuadXor1 = 0xb1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4e;        // quad_perm [2, 3, 0, 1]

__device__ __forceinline__ float wave_sum16(const float (&v)[16], int lane)
{
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = lane_swap_sum32(v[i], v[8 + i]);  // lanes 32..63 hold value 8 + i
    float b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = lane_swap_sum16(a[i], a[4 + i]);  // odd rows hold value 4 + i
    float c[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const bool up = lane & 8;
        const float send = up ? b[i] : b[2 + i];
        c[i] = (up ? b[2 + i] : b[i]) + dpp<kDppRowRor8>(send);
    }
    // lanes 0..3 and 4..7 of each 8-lane group pair up as i and 7 - i
    const bool up = lane & 4;
    float x = (up ? c[1] : c[0]) + dpp<kDppRowHalfMirror>(up ? c[0] : c[1]);
    x += dpp<kDppQuadXor2>(x);
    x += dpp<kDppQuadXor1>(x);
    return x;
}

__device__ __forceinline__ int wave_sum16_index(int lane)
{
    return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}

template <int TW, int TH>
__global__ __launch_bounds__(256) void k_blend_bwd(const uint2 *__restrict__ ranges,
                                                   const uint32_t *__restrict__ work_order,
                                                   const uint32_t *__restrict__ n_items_p,
                                                   const uint32_t *__restrict__ inst_ids,
                                                   const float4 *__restrict__ records,
                                                   const DevView *__restrict__ views, BlendParams P,
                                                   float *__restrict__ record_grads, unsigned int *__restrict__ queue)
{
    constexpr int PPL = slot_layout(TW, TH).slots;
    __shared__ float4 s_rec[4][64][4];
    __shared__ uint32_t s_id[4][64];
    const uint32_t amax_bits = __float_as_uint(P.alpha_max);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nq = min((int)gridDim.x, kQueues), q = (int)blockIdx.x % nq;
    unsigned int *const head = queue + q * kQueueStride;
    const int64_t n_items = *n_items_p;
    for (;;) {
        const int64_t slot = q + (int64_t)nq * wave_fetch_add(head, 1u);
        if (slot >= n_items) break;
        const uint32_t item = work_order[slot];
        const int tile = (int)(item >> 2);
        // pixel slots [k_lo, k_hi) of the lanes: all, or one half of the rows
        const int part = (int)(item & 3u);
        const int k_lo = part == 2 ? PPL / 2 : 0, k_hi = part == 1 ? PPL / 2 : PPL;
        const DevView &V = views[find_view(views, P.n_views, tile)];
        const int local = tile - V.tile_base;
        const int tx = local % V.tiles_x, ty = local / V.tiles_x;
        const int ox = (tx * TW) & ~31, oy = (ty * TH) & ~31;
        const float x0 = (float)ox, y0 = (float)oy;
        const size_t plane = (size_t)V.width * V.height;
        float T[PPL], S[PPL], g0[PPL], g1[PPL], g2[PPL], pxr[PPL], pyr[PPL];
        int last[PPL];
        int maxlast = 0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int px = tx * TW + slot_x<TW, TH>(lane, k), py = ty * TH + slot_y<TW, TH>(lane, k);
            pxr[k] = (float)(px - ox) + 0.5f;
            pyr[k] = (float)(py - oy) + 0.5f;
            T[k] = 1.0f;
            S[k] = 0.0f;
            g0[k] = g1[k] = g2[k] = 0.0f;
            last[k] = 0;
            if (k >= k_lo && k < k_hi && px < V.width && py < V.height) {
                const size_t p = (size_t)py * V.width + px;
                T[k] = V.final_T[p];
                last[k] = V.n_contrib[p];
                g0[k] = V.dL_drgb[p];
                g1[k] = V.dL_drgb[plane + p];
                g2[k] = V.dL_drgb[2 * plane + p];
                S[k] = T[k] * (P.bg0 * g0[k] + P.bg1 * g1[k] + P.bg2 * g2[k]);
                maxlast = max(maxlast, last[k]);
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, d, 64));
        const uint2 rg = ranges[tile];
        maxlast = min(maxlast, (int)(rg.y - rg.x));
        // The last batch of the walked part of the list goes straight to LDS.
        // While a batch is walked back, the raw records of the batch before
        // it and the ids of the one before that are in flight, with no branch
        // around their loads (indices clamped into the list, ids into the
        // record array), so the wait for them falls after the batch.
        uint32_t nid = 0u;
        if (maxlast > 0) {
            const int lo = maxlast > 64 ? maxlast - 64 : 0;
            if (lane < maxlast - lo) {
                const uint32_t v = inst_ids[rg.x + lo + lane];
                const uint32_t id = v & kIdMask;
                s_id[wave][lane] = id < P.n_records ? id : 0xffffffffu;
                float4 r[4];
                fetch_record(r, records, v, P.n_records, PPL <= 4);
                put_test_form(s_rec[wave][lane], r, x0, y0, P.log2_pmin);
            }
            const int nlo = lo > 64 ? lo - 64 : 0;
            nid = inst_ids[rg.x + min(nlo + lane, maxlast - 1)];
        }
        for (int hi = maxlast; hi > 0; hi -= 64) {
            const int lo = hi > 64 ? hi - 64 : 0;
            const int nb = hi - lo;
            const int nlo = lo > 64 ? lo - 64 : 0;
            const bool have_next = lane < lo - nlo;
            const uint32_t cid = nid;
            float4 raw[4];
            PlainModel::load_raw(raw, records, cid, P.n_records);
            const int nnlo = nlo > 64 ? nlo - 64 : 0;
            nid = inst_ids[rg.x + min(nnlo + lane, maxlast - 1)];
            lds_wave_sync();
            for (int jj = nb - 1; jj >= 0; --jj) {
                const int j = lo + jj;
                const TRec R = load_trec(s_rec[wave][jj]);
                const RowSpan span = row_span(R.rows, ty * TH);
                const uint32_t bands = __builtin_amdgcn_readfirstlane(R.rows);
                // the slots of a lane share its pixel column when they are row
                // bands (one slot across)
                constexpr bool one_column = slot_layout(TW, TH).bx == 1;
                const float dx0 = pxr[0] - R.cx;
                // sums over the lane's pixels of dL/dq and its moments in dx
                // and dy, of dL/dden and its moments (q, den, D as in
                // frag_test); the record gradients follow from them once per
                // record (with one column, the dx moments are dx times the
                // plain sums)
                float sq = -0.0f, sqx = -0.0f, sqy = -0.0f, sxx = -0.0f, sxy = -0.0f, syy = -0.0f;
                float sd = -0.0f, sdx = -0.0f, sdy = -0.0f, dic2 = -0.0f, dop = -0.0f;
                float dr = -0.0f, dg = -0.0f, db = -0.0f;
                bool wave_hit = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    if (k < k_lo || k >= k_hi || !band_open<TW, TH>(bands, span, k)) continue;
                    // every lane evaluates the fragment; a lane that does not hit
                    // takes omega = 0 and 1/t = 0, so every term it adds is zero
                    // and its state is unchanged (1 / (1 - 0) = 1 exactly)
                    Frag f;
                    const bool hit = (j < last[k]) & frag_test(R, pxr[k], pyr[k], f);
                    if (__ballot(hit) == 0) continue;
                    wave_hit = true;
                    frag_omega(R, f);
                    const float w = hit ? f.w : 0.0f;
                    const float rt = hit ? f.rt : 0.0f;
                    // omega >= 0, alpha_max > 0: the minimum of the bit patterns
                    const float a = __uint_as_float(min(__float_as_uint(w), amax_bits));
                    const float rom = __builtin_amdgcn_rcpf(1.0f - a);  // 1 / (1 - alpha), alpha <= alpha_max
                    const float Tb = T[k] * rom;  // transmittance in front of this Gaussian
                    const float rgd = __builtin_fmaf(R.b, g2[k], __builtin_fmaf(R.g, g1[k], R.r * g0[k]));
                    const float ta = Tb * a;
                    dr = __builtin_fmaf(ta, g0[k], dr);
                    dg = __builtin_fmaf(ta, g1[k], dg);
                    db = __builtin_fmaf(ta, g2[k], db);
                    const float dL_da = __builtin_fmaf(Tb, rgd, -(S[k] * rom));
                    S[k] = __builtin_fmaf(ta, rgd, S[k]);
                    T[k] = Tb;
                    // alpha clamped at alpha_max passes no gradient to omega
                    const float wd = w < P.alpha_max ? w * dL_da : 0.0f;
                    dop += wd;  // sum of w dL/dw: the record opacity times dL/d(opacity)
                    // dL/dD = -w dL/domega / 2; D = q / t with t = den^2 + q / c^2,
                    // so with ew = w dL/domega / t^2: dL/dq = -ew den^2 / 2,
                    // dL/dden = ew q den, dL/d(1/c^2) = ew q^2 / 2.  The sums
                    // below leave out the constant factors (-1/2 for the q
                    // moments, 1/2 for dic2) and are in the test form's units
                    // (qs = s^2 q): both are applied by the per-Gaussian backward
                    const float ew = wd * (rt * rt);
                    const float dq = ew * (f.den * f.den);
                    const float dden = ew * (f.q * f.den);
                    dic2 = __builtin_fmaf(ew, f.q * f.q, dic2);
                    const float dqy = dq * f.dy;
                    sqy += dqy;
                    syy = __builtin_fmaf(dqy, f.dy, syy);
                    sd += dden;
                    sdy = __builtin_fmaf(dden, f.dy, sdy);
                    if (one_column) {
                        sq += dq;
                    } else {
                        const float dqx = dq * f.dx;
                        sqx += dqx;
                        sxx = __builtin_fmaf(dqx, f.dx, sxx);
                        sxy = __builtin_fmaf(dqx, f.dy, sxy);
                        sdx = __builtin_fmaf(dden, f.dx, sdx);
                    }
                }
                if (!wave_hit) continue;
                if (one_column) {
                    sqx = dx0 * sq;
                    sxx = dx0 * sqx;
                    sxy = dx0 * sqy;
                    sdx = dx0 * sd;
                }
                // the record's gradient as raw sums (layout at kGradFloats);
                // the per-Gaussian backward turns them into dL/d(record) once
                // per Gaussian-view, in double precision, rather than once per
                // (record, tile) here
                const float vals[16] = {sqx, sqy, sxx, sxy, syy, sdx, sdy, sd, dic2, dop, dr,
                                        dg, db, 0.f, 0.f, 0.f};
                const float sum = wave_sum16(vals, lane);
                const int c = wave_sum16_index(lane);
                const uint32_t rid = s_id[wave][jj];
                // one lane per component adds it to the record's accumulators
                if ((lane & 3) == 0 && c < 13 && rid != 0xffffffffu)
                    atomicAdd(record_grads + (size_t)rid * kGradFloats + c, sum);
            }
            lds_wave_sync();
            if (have_next) {
                PlainModel::settle(raw, cid, P.n_records, PPL <= 4);
                put_test_form(s_rec[wave][lane], raw, x0, y0, P.log2_pmin);
                const uint32_t id = cid & kIdMask;
                s_id[wave][lane] = id < P.n_records ? id : 0xffffffffu;
            }
        }
    }
}

// Backward compositing for the exact MIP weight (mip = 2).  The walk is
// that of k_blend_bwd; per fragment, with g = dL/d ln omega (zero for lanes
// that do not hit or whose alpha is clamped) and ln omega =
// ln2 log2o + (ln B - ln den - num / den) / 2 (see ExactMipModel):
//   d/dden = g (num - den) / (2 den^2), d/dnum = -g / (2 den), d/dB = g / (2 B)
//   plus the widening a = E t^2 (E = e / |xbar|, t = A / B), which reaches
//   every S_k = s'_k^2 + a; den = sum q_k prod_{j != k} S_j with q = r^2,
//   num = sum S_k w_k^2, r = rho + P0 dx + P1 dy, w = Q0 dx + Q1 dy,
//   A = sum rho_k r_k / s'_k^2, B = sum r_k^2 / s'_k^2.
// The record gradient (kGradFloatsExactMip floats) is
//   [0, 1] the projected centre, [2..4] P0, [5..7] P1, [8..10] Q0,
//   [11..13] Q1, [14..16] rho, [17..19] s'^2, [20] e, [21] log2o,
//   [22..24] colour.
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_blend_bwd_exact(const uint2 *__restrict__ ranges,
                                                         const uint32_t *__restrict__ work_order,
                                                         const uint32_t *__restrict__ n_items_p,
                                                         const uint32_t *__restrict__ inst_ids,
                                                         const float4 *__restrict__ records,
                                                         const DevView *__restrict__ views, BlendParams P,
                                                         float *__restrict__ record_grads,
                                                         unsigned int *__restrict__ queue)
{
    using M = ExactMipModel;
    constexpr int PPL = slot_layout(TW, TH).slots;
    constexpr float kLn2 = 0.69314718055994531f;
    __shared__ float4 s_rec[4][64][M::kStaged];
    __shared__ uint32_t s_id[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nq = min((int)gridDim.x, kQueues), q = (int)blockIdx.x % nq;
    unsigned int *const head = queue + q * kQueueStride;
    const int64_t n_items = *n_items_p;
    for (;;) {
        const int64_t slot = q + (int64_t)nq * wave_fetch_add(head, 1u);
        if (slot >= n_items) break;
        const uint32_t item = work_order[slot];
        const int tile = (int)(item >> 2);
        const int part = (int)(item & 3u);
        const int k_lo = part == 2 ? PPL / 2 : 0, k_hi = part == 1 ? PPL / 2 : PPL;
        const DevView &V = views[find_view(views, P.n_views, tile)];
        const int local = tile - V.tile_base;
        const int tx = local % V.tiles_x, ty = local / V.tiles_x;
        const int ox = (tx * TW) & ~31, oy = (ty * TH) & ~31;
        const float x0 = (float)ox, y0 = (float)oy;
        const size_t plane = (size_t)V.width * V.height;
        float T[PPL], S[PPL], g0[PPL], g1[PPL], g2[PPL], pxr[PPL], pyr[PPL], aux[PPL];
        int last[PPL];
        int maxlast = 0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int px = tx * TW + slot_x<TW, TH>(lane, k), py = ty * TH + slot_y<TW, TH>(lane, k);
            pxr[k] = (float)(px - ox) + 0.5f;
            pyr[k] = (float)(py - oy) + 0.5f;
            aux[k] = M::pixel_aux(V, px, py);
            T[k] = 1.0f;
            S[k] = 0.0f;
            g0[k] = g1[k] = g2[k] = 0.0f;
            last[k] = 0;
            if (k >= k_lo && k < k_hi && px < V.width && py < V.height) {
                const size_t p = (size_t)py * V.width + px;
                T[k] = V.final_T[p];
                last[k] = V.n_contrib[p];
                g0[k] = V.dL_drgb[p];
                g1[k] = V.dL_drgb[plane + p];
                g2[k] = V.dL_drgb[2 * plane + p];
                S[k] = T[k] * (P.bg0 * g0[k] + P.bg1 * g1[k] + P.bg2 * g2[k]);
                maxlast = max(maxlast, last[k]);
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, d, 64));
        const uint2 rg = ranges[tile];
        maxlast = min(maxlast, (int)(rg.y - rg.x));
        for (int hi = maxlast; hi > 0; hi -= 64) {
            const int lo = hi > 64 ? hi - 64 : 0;
            const int nb = hi - lo;
            if (lane < nb) {
                const uint32_t v = inst_ids[rg.x + lo + lane];
                const uint32_t id = v & kIdMask;
                s_id[wave][lane] = id < P.n_records ? id : 0xffffffffu;
                float4 r[M::kRaw];
                M::fetch(r, records, v, P.n_records, PPL <= 4);
                M::stage(s_rec[wave][lane], r, x0, y0, P.log2_pmin);
            }
            lds_wave_sync();
            for (int jj = nb - 1; jj >= 0; --jj) {
                const int j = lo + jj;
                const XRec R = M::load(s_rec[wave][jj]);
                const RowSpan span = row_span(R.rows, ty * TH);
                const uint32_t bands = __builtin_amdgcn_readfirstlane(R.rows);
                float acc[25];
#pragma unroll
                for (int c = 0; c < 25; ++c) acc[c] = 0.0f;
                bool wave_hit = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    if (k < k_lo || k >= k_hi || !band_open<TW, TH>(bands, span, k)) continue;
                    XFrag f;
                    const bool hit = (j < last[k]) & M::test(R, pxr[k], pyr[k], aux[k], P.log2_pmin, f);
                    if (__ballot(hit) == 0) continue;
                    wave_hit = true;
                    const float w = hit ? M::omega(R, f) : 0.0f;
                    const float a = fminf(w, P.alpha_max);
                    const float rom = __builtin_amdgcn_rcpf(1.0f - a);
                    const float Tb = T[k] * rom;
                    const float rgd = R.r * g0[k] + R.g * g1[k] + R.b * g2[k];
                    const float ta = Tb * a;
                    acc[22] += ta * g0[k];
                    acc[23] += ta * g1[k];
                    acc[24] += ta * g2[k];
                    const float dL_da = Tb * rgd - S[k] * rom;
                    S[k] += ta * rgd;
                    T[k] = Tb;
                    // g = dL / d ln omega; a clamped alpha passes none
                    const float g = (hit & (w < P.alpha_max)) ? dL_da * w : 0.0f;
                    const float rd = hit ? f.rd : 0.0f;
                    const float rB = hit ? f.rB : 0.0f;
                    const float gden = 0.5f * g * (f.num - f.den) * (rd * rd);
                    const float gnum = -0.5f * g * rd;
                    const float gB0 = 0.5f * g * rB;
                    const float gS0 = gden * (f.q1 * f.S2 + f.q2 * f.S1) + gnum * (f.w0 * f.w0);
                    const float gS1 = gden * (f.q0 * f.S2 + f.q2 * f.S0) + gnum * (f.w1 * f.w1);
                    const float gS2 = gden * (f.q0 * f.S1 + f.q1 * f.S0) + gnum * (f.w2 * f.w2);
                    const float ga = gS0 + gS1 + gS2;
                    const float E = R.e * aux[k];
                    const float gt = ga * 2.0f * E * f.t;
                    const float gA = gt * rB;
                    const float gB = gB0 - gt * f.t * rB;
                    const float gr0 = 2.0f * f.r0 * (gden * f.p12 + gB * R.isx) + gA * R.ix_;
                    const float gr1 = 2.0f * f.r1 * (gden * f.p02 + gB * R.isy) + gA * R.iy_;
                    const float gr2 = 2.0f * f.r2 * (gden * f.p01 + gB * R.isz) + gA * R.iz_;
                    const float gw0 = 2.0f * gnum * f.S0 * f.w0;
                    const float gw1 = 2.0f * gnum * f.S1 * f.w1;
                    const float gw2 = 2.0f * gnum * f.S2 * f.w2;
                    acc[0] -= gr0 * R.P0x + gr1 * R.P0y + gr2 * R.P0z + gw0 * R.Q0x + gw1 * R.Q0y + gw2 * R.Q0z;
                    acc[1] -= gr0 * R.P1x + gr1 * R.P1y + gr2 * R.P1z + gw0 * R.Q1x + gw1 * R.Q1y + gw2 * R.Q1z;
                    acc[2] += gr0 * f.dx;
                    acc[3] += gr1 * f.dx;
                    acc[4] += gr2 * f.dx;
                    acc[5] += gr0 * f.dy;
                    acc[6] += gr1 * f.dy;
                    acc[7] += gr2 * f.dy;
                    acc[8] += gw0 * f.dx;
                    acc[9] += gw1 * f.dx;
                    acc[10] += gw2 * f.dx;
                    acc[11] += gw0 * f.dy;
                    acc[12] += gw1 * f.dy;
                    acc[13] += gw2 * f.dy;
                    acc[14] += gr0 + gA * R.isx * f.r0;
                    acc[15] += gr1 + gA * R.isy * f.r1;
                    acc[16] += gr2 + gA * R.isz * f.r2;
                    acc[17] += gS0 - gB * (R.isx * R.isx) * f.q0 - gA * R.rx * (R.isx * R.isx) * f.r0;
                    acc[18] += gS1 - gB * (R.isy * R.isy) * f.q1 - gA * R.ry * (R.isy * R.isy) * f.r1;
                    acc[19] += gS2 - gB * (R.isz * R.isz) * f.q2 - gA * R.rz * (R.isz * R.isz) * f.r2;
                    acc[20] += ga * aux[k] * (f.t * f.t);
                    acc[21] += g * kLn2;
                }
                if (!wave_hit) continue;
                const uint32_t rid = s_id[wave][jj];
                const int c = wave_sum16_index(lane);
                const float lo16[16] = {acc[0], acc[1], acc[2], acc[3], acc[4], acc[5], acc[6], acc[7],
                                        acc[8], acc[9], acc[10], acc[11], acc[12], acc[13], acc[14], acc[15]};
                const float s_lo = wave_sum16(lo16, lane);
                const float hi16[16] = {acc[16], acc[17], acc[18], acc[19], acc[20], acc[21], acc[22], acc[23],
                                        acc[24], 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                const float s_hi = wave_sum16(hi16, lane);
                if ((lane & 3) == 0 && rid != 0xffffffffu) {
                    float *dst = record_grads + (size_t)rid * kGradFloatsExactMip;
                    atomicAdd(dst + c, s_lo);
                    if (c < 9) atomicAdd(dst + 16 + c, s_hi);
                }
            }
            lds_wave_sync();
        }
    }
}

template <int TW, int TH>
int occupancy_grid(const void *kernel, int num_cus)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * num_cus;
}

BlendParams make_params(const DevOptions &opt, int n_views, int64_t total_tiles, int64_t n_records,
                        unsigned long long *item_clock)
{
    return BlendParams{(float)log2(opt.p_min), (float)opt.alpha_max, (float)opt.t_eps, opt.bg[0], opt.bg[1], opt.bg[2],
                       n_views, (int)total_tiles, (uint32_t)n_records, item_clock};
}

// Frame start clock and cleared per-view completion clocks.
__global__ void k_view_clock_start(unsigned long long *__restrict__ stamps, int n_views)
{
    const int i = threadIdx.x;
    if (i == 0) stamps[0] = wall_clock64();
    for (int v = i; v < n_views; v += blockDim.x) stamps[1 + v] = 0ull;
}

// stamps[1 + v] = the latest completion clock over the work items of view v.
__global__ __launch_bounds__(256) void k_view_clock_max(const unsigned long long *__restrict__ item_clock,
                                                         const uint32_t *__restrict__ work_order,
                                                         const uint32_t *__restrict__ n_items_p,
                                                         const DevView *__restrict__ views, int n_views,
                                                         unsigned long long *__restrict__ stamps)
{
    __shared__ unsigned long long best[kMaxViews];
    for (int v = threadIdx.x; v < n_views; v += blockDim.x) best[v] = 0ull;
    __syncthreads();
    const int64_t n_items = *n_items_p;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_items; s += (int64_t)gridDim.x * blockDim.x) {
        const int v = find_view(views, n_views, (int)(work_order[s] >> 2));
        atomicMax(&best[v], item_clock[s]);
    }
    __syncthreads();
    for (int v = threadIdx.x; v < n_views; v += blockDim.x)
        if (best[v]) atomicMax(&stamps[1 + v], best[v]);
}

}  // namespace

bool tile_shape_supported(int w, int h)
{
    return (w == 8 || w == 16 || w == 32) && (h == 8 || h == 16 || h == 32);
}

#define RGS_SHAPES(X) X(8, 8) X(8, 16) X(8, 32) X(16, 8) X(16, 16) X(16, 32) X(32, 8) X(32, 16) X(32, 32)

int blend_grid(TileShape s, bool exact_mip, int num_cus)
{
#define X(W, H)                                                                                                  \
    if (s.w == W && s.h == H)                                                                                    \
        return exact_mip ? occupancy_grid<W, H>(reinterpret_cast<const void *>(&k_blend<W, H, ExactMipModel>), num_cus) \
                         : occupancy_grid<W, H>(reinterpret_cast<const void *>(&k_blend<W, H, PlainModel>), num_cus);
    RGS_SHAPES(X)
#undef X
    return num_cus;
}

int blend_backward_grid(TileShape s, bool exact_mip, int num_cus)
{
#define X(W, H)                                                                                                  \
    if (s.w == W && s.h == H)                                                                                    \
        return exact_mip ? occupancy_grid<W, H>(reinterpret_cast<const void *>(&k_blend_bwd_exact<W, H>), num_cus) \
                         : occupancy_grid<W, H>(reinterpret_cast<const void *>(&k_blend_bwd<W, H>), num_cus);
    RGS_SHAPES(X)
#undef X
    return num_cus;
}

hipError_t launch_blend(TileShape s, const uint2 *ranges, const uint32_t *work_order, const uint32_t *n_items,
                        const uint32_t *inst_ids, const float4 *records, const DevView *views, int n_views,
                        int64_t total_tiles, int64_t n_records, const DevOptions &opt, unsigned int *queue, int grid,
                        unsigned long long *item_clock, hipStream_t stream)
{
    const BlendParams P = make_params(opt, n_views, total_tiles, n_records, item_clock);
#define X(W, H)                                                                                                  \
    if (s.w == W && s.h == H) {                                                                                  \
        if (opt.mip == 2)                                                                                        \
            k_blend<W, H, ExactMipModel><<<grid, 256, 0, stream>>>(ranges, work_order, n_items, inst_ids, records, \
                                                                   views, P, queue);                             \
        else                                                                                                     \
            k_blend<W, H, PlainModel><<<grid, 256, 0, stream>>>(ranges, work_order, n_items, inst_ids, records,   \
                                                                views, P, queue);                                \
        return hipGetLastError();                                                                                \
    }
    RGS_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_blend_backward(TileShape s, const uint2 *ranges, const uint32_t *work_order,
                                 const uint32_t *n_items, const uint32_t *inst_ids, const float4 *records,
                                 const DevView *views, int n_views, int64_t total_tiles, int64_t n_records,
                                 const DevOptions &opt, float *record_grads, unsigned int *queue, int grid,
                                 hipStream_t stream)
{
    const BlendParams P = make_params(opt, n_views, total_tiles, n_records, nullptr);
#define X(W, H)                                                                                                  \
    if (s.w == W && s.h == H) {                                                                                  \
        if (opt.mip == 2)                                                                                        \
            k_blend_bwd_exact<W, H><<<grid, 256, 0, stream>>>(ranges, work_order, n_items, inst_ids, records,    \
                                                              views, P, record_grads, queue);                    \
        else                                                                                                     \
            k_blend_bwd<W, H><<<grid, 256, 0, stream>>>(ranges, work_order, n_items, inst_ids, records, views,   \
                                                        P, record_grads, queue);                                 \
        return hipGetLastError();                                                                                \
    }
    RGS_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_view_clock_start(unsigned long long *stamps, int n_views, hipStream_t stream)
{
    k_view_clock_start<<<1, 256, 0, stream>>>(stamps, n_views);
    return hipGetLastError();
}

hipError_t launch_view_clock_max(const unsigned long long *item_clock, const uint32_t *work_order,
                                 const uint32_t *n_items, int64_t max_items, const DevView *views, int n_views,
                                 unsigned long long *stamps, hipStream_t stream)
{
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_items + 255) / 256, 1024));
    k_view_clock_max<<<grid, 256, 0, stream>>>(item_clock, work_order, n_items, views, n_views, stamps);
    return hipGetLastError();
}

}  // namespace rgs
