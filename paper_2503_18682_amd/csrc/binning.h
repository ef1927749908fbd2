// Exact support-versus-tile test of the emission kernel, in double precision
// on the support conic the preprocess kernel stores per Gaussian-view.
//
// In pixel offsets delta = p - pi(mu) the support omega >= p_min, tau > 0 of a
// Gaussian whose quad lies in front of the camera is the ellipse
//     F(delta) = delta^T P delta - 2 h . delta - f0 <= 0,
// P = b^2 G^T G - kappa g g^T, h = kappa k0 g, f0 = kappa k0^2
// (from q b^2 <= kappa den^2 with q = |G delta|^2, den = k0 + g . delta,
// b^2 = 1 - kappa / c^2).  When P is not positive definite the support is
// unbounded on the image plane and every tile of the bounding rectangle is
// kept.  Tiles are binned from the Gaussian's binning box (binning_clip
// below: the pixels of its pixel box whose centres lie in the ellipse's
// bounding box), and a tile is listed when the continuous rectangle spanned
// by its pixel centres inside the binning box meets the ellipse.  Its
// pixel slots, the 64-pixel groups that a compositing wave tests or skips
// together (slot_layout below), are tested the same way, and the bits of the
// slots that meet the ellipse travel with the instance.  The tests are done
// per tile row: the ellipse's x-extent over the row's heights and over each
// slot row's heights is computed in closed form, then each tile and slot of
// the row is an interval comparison.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rgs {

struct Conic {
    double P00, P01, P11, h0, h1, f0, u0, v0;  // u0, v0: projected centre (pixels)
};

// Pixel box of a Gaussian-view: x0 | x1 << 16, y0 | y1 << 16 (inclusive).
struct PixelBox {
    int x0, x1, y0, y1;
};

__host__ __device__ inline PixelBox unpack_box(uint2 b)
{
    return PixelBox{(int)(b.x & 0xffffu), (int)(b.x >> 16), (int)(b.y & 0xffffu), (int)(b.y >> 16)};
}

// Quantities of the ellipse derived once per Gaussian-view (delta units):
// centre c = P^-1 h, R^2 = f0 + h . c (so the ellipse is
// (d - c)^T P (d - c) <= R^2), its extents and the heights of its leftmost
// and rightmost points.
struct ConicFrame {
    double cx, cy, xmin, xmax, ymin, ymax, yleft, yright, inv_p00;
    bool bounded;
};

__device__ inline ConicFrame conic_frame(const Conic &C)
{
#pragma clang fp contract(off)
    ConicFrame F{};
    const double det = C.P00 * C.P11 - C.P01 * C.P01;
    F.bounded = C.P00 > 0.0 && det > 0.0;
    if (!F.bounded) return F;
    F.cx = (C.P11 * C.h0 - C.P01 * C.h1) / det;
    F.cy = (C.P00 * C.h1 - C.P01 * C.h0) / det;
    const double R2 = C.f0 + C.h0 * F.cx + C.h1 * F.cy;
    const double hx = sqrt(R2 * C.P11 / det), hy = sqrt(R2 * C.P00 / det);
    const double sy = C.P01 * sqrt(R2 / (C.P11 * det));
    F.xmin = F.cx - hx;
    F.xmax = F.cx + hx;
    F.ymin = F.cy - hy;
    F.ymax = F.cy + hy;
    F.yleft = F.cy + sy;
    F.yright = F.cy - sy;
    F.inv_p00 = 1.0 / C.P00;
    return F;
}

// Binning box of a Gaussian-view: the pixels [x0, x1] x [y0, y1] of its pixel
// box [px0, px1] x [py0, py1] whose centres lie in the bounding box of the
// support ellipse, or the pixel box itself when the support is unbounded.
// No pixel centre outside it can hold support, so no tile outside it can be
// listed.  Returns false when it holds no pixel.
__device__ inline bool binning_clip(const Conic &C, int px0, int px1, int py0, int py1, int &x0, int &x1, int &y0,
                                    int &y1)
{
#pragma clang fp contract(off)
    x0 = px0;
    x1 = px1;
    y0 = py0;
    y1 = py1;
    const ConicFrame F = conic_frame(C);
    if (F.bounded) {
        const double ex0 = ceil(C.u0 + F.xmin - 0.5), ex1 = floor(C.u0 + F.xmax - 0.5);
        const double ey0 = ceil(C.v0 + F.ymin - 0.5), ey1 = floor(C.v0 + F.ymax - 0.5);
        if (ex0 > x0) x0 = ex0 > px1 + 1 ? px1 + 1 : (int)ex0;
        if (ex1 < x1) x1 = ex1 < px0 - 1 ? px0 - 1 : (int)ex1;
        if (ey0 > y0) y0 = ey0 > py1 + 1 ? py1 + 1 : (int)ey0;
        if (ey1 < y1) y1 = ey1 < py0 - 1 ? py0 - 1 : (int)ey1;
    }
    return x0 <= x1 && y0 <= y1;
}

// x-extent [xl, xr] of the ellipse over heights y in [ya, yb]; false if the
// ellipse does not reach that height range.  The left boundary is convex and
// the right one concave in y, so off their extreme points the extent is set
// by the chord at an end of the (clipped) range.
__device__ inline bool conic_xrange(const Conic &C, const ConicFrame &F, double ya, double yb, double &xl, double &xr)
{
#pragma clang fp contract(off)
    ya = fmax(ya, F.ymin);
    yb = fmin(yb, F.ymax);
    if (ya > yb) return false;
    const double ys[2] = {ya, yb};
    double lo = INFINITY, hi = -INFINITY;
    for (int e = 0; e < 2; ++e) {
        const double y = ys[e];
        const double bq = C.P01 * y - C.h0;
        const double disc = fmax(bq * bq - C.P00 * (C.P11 * y * y - 2.0 * C.h1 * y - C.f0), 0.0);
        const double r = sqrt(disc);
        lo = fmin(lo, (-bq - r) * F.inv_p00);
        hi = fmax(hi, (-bq + r) * F.inv_p00);
    }
    xl = (F.yleft >= ya && F.yleft <= yb) ? F.xmin : lo;
    xr = (F.yright >= ya && F.yright <= yb) ? F.xmax : hi;
    return true;
}

// Pixel slots of a tile: the compositing kernels give each lane of a wave
// one pixel of every slot, so a slot is 64 pixels that the whole wave skips
// or evaluates together, and a tile's culling bands are its slots.  A tile
// wider than 8 pixels that holds at most 4 blocks of 8 x 8 pixels is cut into
// those blocks (slot k is block (k % bx, k / bx)); any other tile into row
// bands of 64 / TW rows, the full tile width (bx = 1).  Up to 4 slots carry
// per-instance culling bits; a tile with more is tested as one band of TH rows.
struct SlotLayout {
    int bx;     // slots across the tile
    int cw;     // slot width (pixels)
    int rh;     // slot height (pixel rows)
    int slots;  // slots per tile
    bool bits;  // each slot's culling bit travels with the instance
};

__host__ __device__ constexpr SlotLayout slot_layout(int TW, int TH)
{
    return (TW >= 16 && (TW / 8) * (TH / 8) <= 4)
               ? SlotLayout{TW / 8, 8, 8, (TW / 8) * (TH / 8), true}
               : SlotLayout{1, TW, 64 / TW, TH / (64 / TW), TH / (64 / TW) <= 4};
}

constexpr int kMaxBands = 4;

// x-extent of the ellipse, in pixels, over the pixel-centre heights of tile
// row ty (clipped to the box) and over each row band of slots (the rows of
// slot row r = k / bx).
struct BandRanges {
    double row_xl, row_xr;
    double xl[kMaxBands], xr[kMaxBands];
    uint32_t valid;  // slot rows with an extent
    bool row_valid;  // the ellipse reaches the row's heights
};

__device__ inline void band_ranges(const Conic &C, const ConicFrame &F, const PixelBox &box, int ty, int TW, int TH,
                                   BandRanges &B)
{
#pragma clang fp contract(off)
    const SlotLayout S = slot_layout(TW, TH);
    const int nr = S.bits ? S.slots / S.bx : 1, rh = S.bits ? S.rh : TH;  // slot rows
    B.valid = 0u;
    B.row_valid = false;
    B.row_xl = -INFINITY;
    B.row_xr = INFINITY;
    const int y0 = max(ty * TH, box.y0), y1 = min(ty * TH + TH - 1, box.y1);
    if (y0 > y1) return;
    if (!F.bounded)
        B.row_valid = true;
    else
        B.row_valid = conic_xrange(C, F, (double)y0 + 0.5 - C.v0, (double)y1 + 0.5 - C.v0, B.row_xl, B.row_xr);
#pragma unroll
    for (int r = 0; r < kMaxBands; ++r) {
        B.xl[r] = -INFINITY;
        B.xr[r] = INFINITY;
        if (r >= nr || !B.row_valid) continue;
        const int r0 = max(ty * TH + r * rh, box.y0), r1 = min(ty * TH + r * rh + rh - 1, box.y1);
        if (r0 > r1) continue;
        if (!F.bounded) {
            B.valid |= 1u << r;
            continue;
        }
        if (nr == 1) {  // the slot row is the tile row
            B.valid |= 1u;
            B.xl[0] = B.row_xl;
            B.xr[0] = B.row_xr;
            continue;
        }
        double xl, xr;
        if (conic_xrange(C, F, (double)r0 + 0.5 - C.v0, (double)r1 + 0.5 - C.v0, xl, xr)) {
            B.valid |= 1u << r;
            B.xl[r] = xl;
            B.xr[r] = xr;
        }
    }
}

// Is tile (tx, .) of the row listed: does its pixel-centre rectangle (clipped
// to the box) overlap the row's x-extent?  *bands receives the slots whose
// own pixel-centre rectangles overlap their slot row's extent (0 for a tile
// not listed).
__device__ inline bool tile_listed(const Conic &C, const BandRanges &B, const PixelBox &box, int tx, int TW, int TH,
                                   uint32_t &bands)
{
#pragma clang fp contract(off)
    bands = 0u;
    const int cx0 = max(tx * TW, box.x0), cx1 = min(tx * TW + TW - 1, box.x1);
    if (cx0 > cx1 || !B.row_valid) return false;
    const double xa = (double)cx0 + 0.5 - C.u0, xb = (double)cx1 + 0.5 - C.u0;
    if (!(xa <= B.row_xr && xb >= B.row_xl)) return false;
    const SlotLayout S = slot_layout(TW, TH);
    const int nslots = S.bits ? S.slots : 1, bx = S.bits ? S.bx : 1, cw = S.bits ? S.cw : TW;
    // Slot row r and column c are loop constants, so B's arrays stay in
    // registers (a run-time index would put them in scratch memory).
#pragma unroll
    for (int r = 0; r < kMaxBands; ++r) {
#pragma unroll
        for (int c = 0; c < kMaxBands; ++c) {
            const int k = r * bx + c;
            if (c >= bx || k >= nslots) continue;
            const int sx0 = max(tx * TW + c * cw, box.x0), sx1 = min(tx * TW + c * cw + cw - 1, box.x1);
            if (sx0 > sx1 || !((B.valid >> r) & 1u)) continue;
            const double sa = (double)sx0 + 0.5 - C.u0, sb = (double)sx1 + 0.5 - C.u0;
            if (sa <= B.xr[r] && sb >= B.xl[r]) bands |= 1u << k;
        }
    }
    return true;
}

// Instance values carry the culling bits of their tile's slots in the top 4
// bits (a tile with more slots carries none; its rows are then bounded by
// the record's pixel rows).
constexpr uint32_t kIdBits = 28;
constexpr uint32_t kIdMask = (1u << kIdBits) - 1u;

__device__ inline uint32_t pack_instance(uint32_t id, uint32_t bands, int TW, int TH)
{
    return slot_layout(TW, TH).bits ? id | (bands << kIdBits) : id;
}

}  // namespace rgs
