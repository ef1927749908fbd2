// Per Gaussian-view stage: activation, camera transform, culling, MIP
// transform, the 3D bounding quad, its pixel/tile rectangle, the depth key and
// the raster record consumed by the compositing kernel.
//
// One thread per Gaussian loops over the views of the batch, so the
// parameters (236 B per Gaussian at SH degree 3) are read from HBM once per
// batch with coalesced structure-of-arrays loads.  Everything up to the tile
// rectangle and the depth key is evaluated in double precision (full rate on
// CDNA) with FMA contraction disabled, so the integer decisions (culls, tile
// rectangles, keys) are those of an exact evaluation up to double rounding.
#include <hip/hip_fp16.h>

#include "binning.h"
#include "internal.h"
#include "sh.h"

#pragma clang fp contract(off)

namespace rgs {
namespace {

// Exact MIP record (mip = 2; layout and per-ray arithmetic in blend.hip):
// the Gaussian in its own axes with its variances divided by lam = s_max^2.
__device__ void write_exact_mip_record(float4 *rec, const double mu[3], const double Rp[9], const double s[3],
                                       double o, double sig2, const DevView &V, float u_hi, float v_hi,
                                       uint32_t lo_bits, uint32_t rows)
{
    const double smax = fmax(s[0], fmax(s[1], s[2]));
    const double ilam = 1.0 / (smax * smax), iz = 1.0 / mu[2];
    const double u0 = mu[0] * iz, v0 = mu[1] * iz;
    const double qx = mu[2] / (V.fx * smax), qy = mu[2] / (V.fy * smax);
    const double ifx = V.ifx, ify = V.ify;
    double P0[3], P1[3], Q0[3], Q1[3], rho[3], s2[3];
    for (int k = 0; k < 3; ++k) {
        // (R_p^T e_r)_k = R_p[r][k]
        P0[k] = Rp[k] * ifx;
        P1[k] = Rp[3 + k] * ify;
        Q0[k] = (Rp[3 + k] - v0 * Rp[6 + k]) * qx;
        Q1[k] = (u0 * Rp[6 + k] - Rp[k]) * qy;
        rho[k] = (Rp[k] * mu[0] + Rp[3 + k] * mu[1] + Rp[6 + k] * mu[2]) * iz;
        s2[k] = s[k] * s[k] * ilam;
    }
    const double e = sig2 * mu[2] * mu[2] * ilam;
    const double log2o = log2(o) + 0.5 * log2(s2[0] * s2[1] * s2[2]);
    rec[0] = make_float4(u_hi, v_hi, __uint_as_float(lo_bits), __uint_as_float(rows));
    rec[1] = make_float4((float)P0[0], (float)P0[1], (float)P0[2], (float)e);
    rec[2] = make_float4((float)P1[0], (float)P1[1], (float)P1[2], (float)log2o);
    // the fourth floats of rows 3..5 hold the colour (written by colour_view)
    float *f = reinterpret_cast<float *>(rec);
    for (int k = 0; k < 3; ++k) {
        f[12 + k] = (float)Q0[k];
        f[16 + k] = (float)Q1[k];
        f[20 + k] = (float)rho[k];
    }
    rec[6] = make_float4((float)s2[0], (float)s2[1], (float)s2[2], 0.0f);
}

// Projected centre pi(mu) in pixels as a (hi, lo) float pair, lo as fp16 bits
// (|lo| <= half an fp32 ulp of the centre, so fp16 keeps it to ~1e-7 px).
struct Centre {
    double u, v;
    float u_hi, v_hi;
    uint32_t lo_bits;
};

__device__ inline Centre projected_centre(const double mu[3], const DevView &V)
{
    Centre c;
    const double k0 = 1.0 / mu[2];
    c.u = V.fx * mu[0] * k0 + V.cx;
    c.v = V.fy * mu[1] * k0 + V.cy;
    c.u_hi = (float)c.u;
    c.v_hi = (float)c.v;
    const __half2 lo = __floats2half2_rn((float)(c.u - (double)c.u_hi), (float)(c.v - (double)c.v_hi));
    c.lo_bits = *reinterpret_cast<const uint32_t *>(&lo);
    return c;
}


// Kernel variants by divergence and MIP mode, so that each carries only its
// own code (fewer registers and instructions in the common ray-based one).
enum PrepMode { kPrepRay = 0, kPrepMipApprox = 1, kPrepMipExact = 2, kPrepGS = 3 };

// View-dependent colour, max(0, SH(direction camera centre -> mean) + 1/2),
// in two steps.  sh_load keeps Gaussian i's coefficients in the block's LDS
// (coefficient k of thread t at lds[k][t]: each thread only touches its own
// column, and consecutive threads hit consecutive banks) and returns whether
// they are all finite (if not, the Gaussian is culled in every view).
// colour_view then evaluates one view's colour from them into the record's
// colour floats next to the geometry of that view, which writes the rest of
// the record: the two partial writes of a record line follow each other
// closely and merge in L2.  Views that end up culled mostly cost no colour
// (see the view loop of k_preprocess).  The coefficients are read from HBM
// once per batch; they are not held in registers across the FP64 geometry,
// which keeps its occupancy.
template <int DEG>
__device__ __forceinline__ bool sh_load(const float *__restrict__ sh, int n, int i, float (*lds)[256])
{
    constexpr int NK = (DEG + 1) * (DEG + 1);
    bool sh_ok = true;
#pragma unroll
    for (int k = 0; k < NK * 3; ++k) {
        const float c = sh[(size_t)k * n + i];
        lds[k][threadIdx.x] = c;
        sh_ok = sh_ok && isfinite(c);
    }
    return sh_ok;
}

template <int DEG>
__device__ __forceinline__ void colour_view(const float (*lds)[256], const double (&m)[3], const DevView &V,
                                            float *__restrict__ rc, ColourSlot slot)
{
    constexpr int NK = (DEG + 1) * (DEG + 1);
    float c[NK * 3], dir[3], Y[NK], col[3];
#pragma unroll
    for (int k = 0; k < NK * 3; ++k) c[k] = lds[k][threadIdx.x];
    double dist;
    view_dir(m, V.centre, dir, &dist);
    sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
    sh_colour<DEG>(Y, c, col);
#pragma unroll
    for (int k = 0; k < 3; ++k) rc[k * slot.step] = fmaxf(col[k], 0.0f);
    // keep the scheduler from interleaving this with the view's geometry:
    // the colour's temporaries then die before the FP64 registers are needed
    __builtin_amdgcn_sched_barrier(0);
}

template <int MODE, int DEG>
__global__ __launch_bounds__(256) void k_preprocess(const float *__restrict__ means,
                                                    const float *__restrict__ log_scales,
                                                    const float *__restrict__ quats,
                                                    const float *__restrict__ opacity_logits,
                                                    const float *__restrict__ sh, int n,
                                                    const DevView *__restrict__ views, int n_views, DevOptions opt,
                                                    float4 *__restrict__ records, uint32_t *__restrict__ depth_keys,
                                                    uint2 *__restrict__ boxes, uint2 *__restrict__ bin_boxes,
                                                    Conic *__restrict__ conics, uint32_t *__restrict__ tile_counts,
                                                    double *__restrict__ crossing,
                                                    unsigned long long *__restrict__ crossing_count,
                                                    uint32_t crossing_cap)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;

    __shared__ float sh_lds[(DEG + 1) * (DEG + 1) * 3][256];
    const double m[3] = {means[i], means[n + i], means[2 * n + i]};
    const bool sh_ok = sh_load<DEG>(sh, n, i, sh_lds);
    constexpr int rec_floats = MODE == kPrepMipExact ? kRecordFloatsExactMip : kRecordFloats;
    constexpr ColourSlot slot = colour_slot(MODE == kPrepMipExact ? 2 : 0);
    const float lf[3] = {log_scales[i], log_scales[n + i], log_scales[2 * n + i]};
    const float qf[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
    const float af = opacity_logits[i];
    bool ok = sh_ok && isfinite(af);
#pragma unroll
    for (int k = 0; k < 3; ++k) ok = ok && isfinite((float)m[k]) && isfinite(lf[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) ok = ok && isfinite(qf[k]);
    const double q[4] = {qf[0], qf[1], qf[2], qf[3]};
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    ok = ok && qn > 0.0;

    // Sigma = R S^2 R^T in the world frame: rotation of the unit quaternion,
    // s = exp(l), prior opacity o = sigmoid(a).
    // Divisions are taken as products with one reciprocal wherever a value is
    // divided more than once: a double division is a long instruction sequence,
    // and the extra rounding (a few units in the last place of a double) is
    // far below every decision margin of the integer outputs.
    double R[9], s[3], is[3], o = 0.0;
    {
        const double iq = 1.0 / qn;
        const double w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
        R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
        R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
        R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
        for (int k = 0; k < 3; ++k) {
            s[k] = exp((double)lf[k]);
            is[k] = 1.0 / s[k];
        }
        o = 1.0 / (1.0 + exp(-(double)af));
    }
    // support cut-off (eq. 3) and the record's log2 opacity; the MIP transform
    // changes the opacity per view and recomputes them
    const double kappa_o = -2.0 * log(opt.p_min / o);
    const float log2o_o = (float)log2(o);

    for (int v = 0; v < n_views; ++v) {
        const DevView &V = views[v];
        const size_t idx = (size_t)v * n + i;
        uint32_t key = 0xffffffffu, cnt = 0;
        uint2 box = make_uint2(0u, 0u), bin = make_uint2(0u, 0u);
        const double *W = V.w2c;
        // camera-frame centre
        const double mu[3] = {W[0] * m[0] + W[1] * m[1] + W[2] * m[2] + W[3],
                              W[4] * m[0] + W[5] * m[1] + W[6] * m[2] + W[7],
                              W[8] * m[0] + W[9] * m[1] + W[10] * m[2] + W[11]};
        float *const rc = reinterpret_cast<float *>(records) + idx * rec_floats + slot.first;
        // A view whose centre projects inside the image is almost always
        // kept: its colour is evaluated before the geometry (the scheduler
        // then overlaps it best); any other kept view gets it afterwards.
        bool coloured = false;
        if (ok && mu[2] > opt.near_z) {
            const double ux = V.fx * mu[0] + V.cx * mu[2], vy = V.fy * mu[1] + V.cy * mu[2];
            if (ux >= 0.0 && ux <= V.width * mu[2] && vy >= 0.0 && vy <= V.height * mu[2]) {
                colour_view<DEG>(sh_lds, m, V, rc, slot);
                coloured = true;
            }
        }
        do {
            if (!ok || !(mu[2] > opt.near_z)) break;
            double Rp[9];  // R_p = W_rot R
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    Rp[3 * r + c] = W[4 * r] * R[c] + W[4 * r + 1] * R[3 + c] + W[4 * r + 2] * R[6 + c];
            double sv[3] = {s[0], s[1], s[2]}, isv[3] = {is[0], is[1], is[2]};
            double kappa = kappa_o;
            float log2o = log2o_o;
            double ml[3];  // R_p^T mu: centre in the Gaussian's own axes
            for (int c = 0; c < 3; ++c) ml[c] = Rp[c] * mu[0] + Rp[3 + c] * mu[1] + Rp[6 + c] * mu[2];
            if constexpr (MODE == kPrepGS) {
                // Linearised divergence (Sec. 3.1): the pixel-space Gaussian of
                // covariance Sigma_pi = J Sigma J^T, J the Jacobian of the
                // projection at mu; support D_gs <= kappa, an ellipse bounded
                // by its axis-aligned box.  Its record is the plain one with
                // den = 1 (k0 = 1, g = 0, 1/c^2 = 0) and G the Cholesky factor
                // of Sigma_pi^-1, so the compositing kernel evaluates
                // q = |G delta|^2 = D_gs.
                if (!(kappa > 0.0)) break;
                const double iz = 1.0 / mu[2];
                const double J0[3] = {V.fx * iz, 0.0, -V.fx * mu[0] * iz * iz};
                const double J1[3] = {0.0, V.fy * iz, -V.fy * mu[1] * iz * iz};
                double M0[3], M1[3];  // J R_p S
                for (int c = 0; c < 3; ++c) {
                    M0[c] = (J0[0] * Rp[c] + J0[1] * Rp[3 + c] + J0[2] * Rp[6 + c]) * sv[c];
                    M1[c] = (J1[0] * Rp[c] + J1[1] * Rp[3 + c] + J1[2] * Rp[6 + c]) * sv[c];
                }
                const double P00 = M0[0] * M0[0] + M0[1] * M0[1] + M0[2] * M0[2];
                const double P01 = M0[0] * M1[0] + M0[1] * M1[1] + M0[2] * M1[2];
                const double P11 = M1[0] * M1[0] + M1[1] * M1[1] + M1[2] * M1[2];
                const double det = P00 * P11 - P01 * P01;
                if (!(det > 0.0)) break;
                const double idet = 1.0 / det;
                const double A00 = P11 * idet, A01 = -P01 * idet, A11 = P00 * idet;
                const Centre pc = projected_centre(mu, V);
                const double eu = sqrt(kappa * P00), ev = sqrt(kappa * P11);
                const int Wd = V.width, Hd = V.height;
                const double fx0 = ceil(pc.u - eu - 0.5), fx1 = floor(pc.u + eu - 0.5);
                const double fy0 = ceil(pc.v - ev - 0.5), fy1 = floor(pc.v + ev - 0.5);
                const int px0 = fx0 < 0.0 ? 0 : (fx0 > Wd ? Wd : (int)fx0);
                const int px1 = fx1 > Wd - 1 ? Wd - 1 : (fx1 < -1.0 ? -1 : (int)fx1);
                const int py0 = fy0 < 0.0 ? 0 : (fy0 > Hd ? Hd : (int)fy0);
                const int py1 = fy1 > Hd - 1 ? Hd - 1 : (fy1 < -1.0 ? -1 : (int)fy1);
                if (px0 > px1 || py0 > py1) break;
                box = make_uint2((uint32_t)px0 | ((uint32_t)px1 << 16), (uint32_t)py0 | ((uint32_t)py1 << 16));
                bin = box;  // the box is already the support ellipse's
                key = __float_as_uint((float)mu[2]);
                cnt = (uint32_t)(((px1 >> opt.tile_wshift) - (px0 >> opt.tile_wshift) + 1) * ((py1 >> opt.tile_hshift) - (py0 >> opt.tile_hshift) + 1));
                const double G00 = sqrt(A00), G01 = A01 / G00, G11 = sqrt(A11 - G01 * G01);
                float4 *rec = records + idx * 4;
                rec[0] = make_float4(pc.u_hi, pc.v_hi, __uint_as_float(pc.lo_bits),
                                     __uint_as_float((uint32_t)py0 | ((uint32_t)py1 << 16)));
                rec[1] = make_float4((float)G00, (float)G01, 0.0f, (float)G11);
                rec[2] = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
                reinterpret_cast<float *>(rec)[12] = log2o;  // floats 13..15: colour_view's
                conics[idx] = Conic{A00, A01, A11, 0.0, 0.0, kappa, pc.u, pc.v};
                break;
            }
            bool whole = false;  // exact MIP without a bounding Gaussian
            if constexpr (MODE == kPrepMipExact) {
                // Exact MIP: the camera-inside skip applies to the Gaussian
                // itself; the quad, box and tiles are those of the Gaussian
                // widened by a_max = sigma^2 tau_max^2, which bounds the
                // per-ray widening sigma_x^2 tau(x)^2 of every ray that can
                // reach p_min (m <= 1): |tau| <= (|mu| + sqrt(kappa) s_max
                // (1 + rho)) / (1 - beta), rho = s_max / s_min, beta =
                // sqrt(kappa) sigma (1 + rho).  Without such a bound (beta >= 1,
                // or the widened Gaussian holds the camera) the whole view is
                // listed.
                if (!(kappa > 0.0)) break;
                double c2g = 0.0;
                for (int k = 0; k < 3; ++k) c2g += ml[k] * ml[k] * (isv[k] * isv[k]);
                if (!(c2g > kappa)) break;
                const double sig2 = opt.mip_sigma2_px / (V.fx * V.fy);
                const double smax = fmax(sv[0], fmax(sv[1], sv[2])), smin = fmin(sv[0], fmin(sv[1], sv[2]));
                const double rho = smax / smin;
                const double beta = sqrt(kappa * sig2) * (1.0 + rho);
                whole = !(beta < 1.0);
                if (!whole) {
                    const double tb = sqrt(mu[0] * mu[0] + mu[1] * mu[1] + mu[2] * mu[2]);
                    const double tmax = (tb + sqrt(kappa) * smax * (1.0 + rho)) / (1.0 - beta);
                    const double amax = sig2 * tmax * tmax;
                    double sh2[3], c2b = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        sh2[k] = sv[k] * sv[k] + amax;
                        c2b += ml[k] * ml[k] / sh2[k];
                    }
                    whole = !(c2b > kappa);
                    if (!whole)
                        for (int k = 0; k < 3; ++k) {
                            sv[k] = sqrt(sh2[k]);
                            isv[k] = 1.0 / sv[k];
                        }
                }
                if (whole) {
                    const int Wd = V.width, Hd = V.height;
                    box = make_uint2((uint32_t)(Wd - 1) << 16, (uint32_t)(Hd - 1) << 16);
                    bin = box;
                    key = __float_as_uint((float)mu[2]);
                    cnt = (uint32_t)((((Wd - 1) >> opt.tile_wshift) + 1) * (((Hd - 1) >> opt.tile_hshift) + 1));
                    const Centre pc = projected_centre(mu, V);
                    write_exact_mip_record(records + idx * (kRecordFloatsExactMip / 4), mu, Rp, s, o, sig2, V,
                                           pc.u_hi, pc.v_hi, pc.lo_bits, (uint32_t)(Hd - 1) << 16);
                    // P00 = 0: not an ellipse, so every tile of the box is listed
                    conics[idx] = Conic{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, pc.u, pc.v};
                    break;
                }
            } else if constexpr (MODE == kPrepMipApprox) {
                // Approximate MIP (Sec. 5, eq. 17): add sigma^2 |mu|^2 to every
                // variance (pixel-invariant tau = |mu|) and scale the opacity by
                // sqrt(|Sigma| c^2 / (|Sigma^| c^^2)).
                const double tb = sqrt(mu[0] * mu[0] + mu[1] * mu[1] + mu[2] * mu[2]);
                const double sig2 = opt.mip_sigma2_px / (V.fx * V.fy);
                double det = 1.0, deth = 1.0, c2p = 0.0, c2h = 0.0, sh2[3], ish2[3];
                for (int k = 0; k < 3; ++k) {
                    const double s2 = sv[k] * sv[k];
                    sh2[k] = s2 + sig2 * tb * tb;
                    ish2[k] = 1.0 / sh2[k];
                    det *= s2;
                    deth *= sh2[k];
                    c2p += ml[k] * ml[k] * (isv[k] * isv[k]);
                    c2h += ml[k] * ml[k] * ish2[k];
                }
                // mip = 3: the widening without the modulation (dilation only)
                const double ov = opt.mip == 3 ? o : o * sqrt(det * c2p / (deth * c2h));
                for (int k = 0; k < 3; ++k) {
                    sv[k] = sqrt(sh2[k]);
                    isv[k] = sv[k] * ish2[k];
                }
                kappa = -2.0 * log(opt.p_min / ov);
                log2o = (float)log2(ov);
            }
            // support cut-off (eq. 3) and the camera-inside skip (eq. 6)
            if (!(kappa > 0.0)) break;
            const double mw[3] = {ml[0] * isv[0], ml[1] * isv[1], ml[2] * isv[2]};
            const double c2 = mw[0] * mw[0] + mw[1] * mw[1] + mw[2] * mw[2];
            if (!(c2 > kappa)) break;

            // Sec. 4.1: whitened unit centre, b, R_{mu^ <- v} (App. A.1)
            const double c = sqrt(c2);
            const double ic = 1.0 / c, ic2 = 1.0 / c2;
            const double muh[3] = {mw[0] * ic, mw[1] * ic, mw[2] * ic};
            const double b = sqrt(1.0 - kappa * ic2);
            double Rv[9];
            {
                const double sgn = muh[2] >= 0.0 ? 1.0 : -1.0;  // align to v or to -v
                const double a3[3] = {muh[0], muh[1], muh[2] + sgn};
                const double a2 = a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2];
                const double t2 = 2.0 / a2;
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) Rv[3 * r + cc] = t2 * a3[r] * a3[cc] - (r == cc ? 1.0 : 0.0);
                if (sgn < 0.0)  // right-multiply by P = diag(-1, 1, -1)
                    for (int r = 0; r < 3; ++r) {
                        Rv[3 * r] = -Rv[3 * r];
                        Rv[3 * r + 2] = -Rv[3 * r + 2];
                    }
            }
            // Q = R_p S R_v, B = Q_{0:2}^T Q_{0:2} (eq. 14)
            double Q[9];
            for (int r = 0; r < 3; ++r)
                for (int cc = 0; cc < 3; ++cc)
                    Q[3 * r + cc] = (Rp[3 * r] * sv[0]) * Rv[cc] + (Rp[3 * r + 1] * sv[1]) * Rv[3 + cc] +
                                    (Rp[3 * r + 2] * sv[2]) * Rv[6 + cc];
            double Ba = 0.0, Bh = 0.0, Bd = 0.0;
            for (int r = 0; r < 3; ++r) {
                Ba += Q[3 * r] * Q[3 * r];
                Bh += Q[3 * r] * Q[3 * r + 1];
                Bd += Q[3 * r + 1] * Q[3 * r + 1];
            }
            // closed-form top eigenvector u1 of the 2x2 B; u0 = u1 turned by +90 degrees
            const double mean = 0.5 * (Ba + Bd);
            const double rad = sqrt(0.25 * (Ba - Bd) * (Ba - Bd) + Bh * Bh);
            const double lmax = mean + rad;
            double u1x = 1.0, u1y = 0.0;
            if (!(2.0 * rad <= 1e-6 * lmax)) {
                const double v1x = Bh, v1y = lmax - Ba, v2x = lmax - Bd, v2y = Bh;
                const double n1 = sqrt(v1x * v1x + v1y * v1y), n2 = sqrt(v2x * v2x + v2y * v2y);
                const bool first = n1 >= n2;
                const double inv = 1.0 / (first ? n1 : n2);
                u1x = (first ? v1x : v2x) * inv;
                u1y = (first ? v1y : v2y) * inv;
            }
            const double u0x = -u1y, u0y = u1x;
            // quad vertices V_k = mu + Q_{0:2} U (sqrt(kappa)/b) O_k (eq. 15)
            const double hs = sqrt(kappa) / b;
            double QU[6];
            for (int r = 0; r < 3; ++r) {
                QU[2 * r] = Q[3 * r] * u0x + Q[3 * r + 1] * u0y;
                QU[2 * r + 1] = Q[3 * r] * u1x + Q[3 * r + 1] * u1y;
            }
            const double O0[4] = {-1.0, -1.0, 1.0, 1.0}, O1[4] = {-1.0, 1.0, 1.0, -1.0};
            bool all_front = true;
            for (int k = 0; k < 4; ++k)
                if (!(QU[4] * (hs * O0[k]) + QU[5] * (hs * O1[k]) + mu[2] > 0.0)) all_front = false;
            // A vertex at z <= 0 makes the box the whole view here; the quad
            // goes to the crossing list, whose kernel bounds the box by the
            // part of the quad inside the view frustum.
            if (!all_front) {
                const unsigned long long slot = atomicAdd(crossing_count, 1ull);
                if (slot < crossing_cap) {
                    double *e = crossing + slot * kCrossingDoubles;
                    e[0] = mu[0];
                    e[1] = mu[1];
                    e[2] = mu[2];
                    for (int k = 0; k < 6; ++k) e[3 + k] = QU[k];
                    e[9] = hs;
                    e[10] = (double)idx;
                    e[11] = 0.0;
                }
            }
            double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
            for (int k = 0; k < 4; ++k) {
                const double z0 = hs * O0[k], z1 = hs * O1[k];
                const double Vx = QU[0] * z0 + QU[1] * z1 + mu[0];
                const double Vy = QU[2] * z0 + QU[3] * z1 + mu[1];
                const double Vz = QU[4] * z0 + QU[5] * z1 + mu[2];
                const double iz = 1.0 / Vz;
                const double u = V.fx * Vx * iz + V.cx;
                const double vv = V.fy * Vy * iz + V.cy;
                umin = fmin(umin, u);
                umax = fmax(umax, u);
                vmin = fmin(vmin, vv);
                vmax = fmax(vmax, vv);
            }
            // pixel centres inside the box
            const int Wd = V.width, Hd = V.height;
            int px0 = 0, px1 = Wd - 1, py0 = 0, py1 = Hd - 1;
            if (all_front) {
                const double fx0 = ceil(umin - 0.5), fx1 = floor(umax - 0.5);
                const double fy0 = ceil(vmin - 0.5), fy1 = floor(vmax - 0.5);
                px0 = fx0 < 0.0 ? 0 : (fx0 > Wd ? Wd : (int)fx0);
                px1 = fx1 > Wd - 1 ? Wd - 1 : (fx1 < -1.0 ? -1 : (int)fx1);
                py0 = fy0 < 0.0 ? 0 : (fy0 > Hd ? Hd : (int)fy0);
                py1 = fy1 > Hd - 1 ? Hd - 1 : (fy1 < -1.0 ? -1 : (int)fy1);
            }
            if (px0 > px1 || py0 > py1) break;
            box = make_uint2((uint32_t)px0 | ((uint32_t)px1 << 16), (uint32_t)py0 | ((uint32_t)py1 << 16));
            key = __float_as_uint((float)mu[2]);

            // ---- raster record (float32) ----
            const Centre pc = projected_centre(mu, V);
            const double k0 = 1.0 / mu[2];
            const double u_c = pc.u, v_c = pc.v;
            // A2 = (S^-1 R_p^T)[:, 0:2] diag(1/fx, 1/fy): a pixel offset delta moves
            // the whitened ray direction by A2 delta.
            double A2[3][2];
            const double ifx = V.ifx, ify = V.ify;
            for (int k = 0; k < 3; ++k) {
                A2[k][0] = Rp[k] * isv[k] * ifx;
                A2[k][1] = Rp[3 + k] * isv[k] * ify;
            }
            // G = R_v[:, 0:2]^T A2 maps delta to the quad-plane offset (times den)
            double G[2][2];
            for (int r = 0; r < 2; ++r)
                for (int cc = 0; cc < 2; ++cc)
                    G[r][cc] = Rv[r] * A2[0][cc] + Rv[3 + r] * A2[1][cc] + Rv[6 + r] * A2[2][cc];
            const double gx = (A2[0][0] * mw[0] + A2[1][0] * mw[1] + A2[2][0] * mw[2]) * ic2;
            const double gy = (A2[0][1] * mw[0] + A2[1][1] * mw[1] + A2[2][1] * mw[2]) * ic2;
            // support ellipse in pixel offsets; the emission lists the tiles it meets
            Conic C;
            {
                const double M00 = G[0][0] * G[0][0] + G[1][0] * G[1][0];
                const double M01 = G[0][0] * G[0][1] + G[1][0] * G[1][1];
                const double M11 = G[0][1] * G[0][1] + G[1][1] * G[1][1];
                C.P00 = b * b * M00 - kappa * gx * gx;
                C.P01 = b * b * M01 - kappa * gx * gy;
                C.P11 = b * b * M11 - kappa * gy * gy;
                C.h0 = kappa * k0 * gx;
                C.h1 = kappa * k0 * gy;
                C.f0 = kappa * k0 * k0;
                C.u0 = u_c;
                C.v0 = v_c;
            }
            // (written before any cull below: the crossing kernel reads it)
            conics[idx] = C;
            // binning box: the pixels of the box whose centres lie in the
            // support ellipse's bounding box (no tile outside it can be listed)
            int bx0 = px0, bx1 = px1, by0 = py0, by1 = py1;
            if (!binning_clip(C, px0, px1, py0, py1, bx0, bx1, by0, by1)) break;
            bin = make_uint2((uint32_t)bx0 | ((uint32_t)bx1 << 16), (uint32_t)by0 | ((uint32_t)by1 << 16));
            // tiles of the binning box; the emission kernel lists those whose
            // pixel-centre rectangle meets the support and marks the others empty
            cnt = (uint32_t)(((bx1 >> opt.tile_wshift) - (bx0 >> opt.tile_wshift) + 1) * ((by1 >> opt.tile_hshift) - (by0 >> opt.tile_hshift) + 1));
            // the residuals of the centre go into one fp16 pair; the freed slot
            // holds the binning box's pixel rows for in-tile culling
            const uint32_t rows = (uint32_t)by0 | ((uint32_t)by1 << 16);
            if constexpr (MODE == kPrepMipExact) {
                write_exact_mip_record(records + idx * (kRecordFloatsExactMip / 4), mu, Rp, s, o,
                                       opt.mip_sigma2_px / (V.fx * V.fy), V, pc.u_hi, pc.v_hi, pc.lo_bits, rows);
            } else {
                float4 *rec = records + idx * 4;
                rec[0] = make_float4(pc.u_hi, pc.v_hi, __uint_as_float(pc.lo_bits), __uint_as_float(rows));
                rec[1] = make_float4((float)G[0][0], (float)G[0][1], (float)G[1][0], (float)G[1][1]);
                rec[2] = make_float4((float)gx, (float)gy, (float)k0, (float)ic2);
                reinterpret_cast<float *>(rec)[12] = log2o;  // floats 13..15: colour_view's
            }
        } while (false);
        // culled views' records are never read
        if (cnt && !coloured) colour_view<DEG>(sh_lds, m, V, rc, slot);
        depth_keys[idx] = cnt ? key : 0xffffffffu;
        tile_counts[idx] = cnt;
        boxes[idx] = box;
        bin_boxes[idx] = bin;
    }
}

// Box of a quad with a vertex at z <= 0 (Sec. 4.1 draws the quad unclipped;
// only its pixel box is bounded here): the quad, rebuilt from its crossing
// list entry with the arithmetic of the geometry kernel, is clipped
// (Sutherland-Hodgman) against the four side planes of the view frustum,
// which pass through the camera centre and the image borders; the box is
// that of the projected clipped polygon.  No part inside: the Gaussian-view
// is culled.  A clipped vertex at z <= 0 (only the camera centre can be one),
// or a polygon beyond kClipMaxVerts vertices (rounding only), keeps the
// whole view.  One wave per block; each lane keeps its two polygons in LDS.
constexpr int kClipBlock = 64, kClipMaxVerts = 16, kClipGrid = 32;

__global__ __launch_bounds__(kClipBlock) void k_clip_crossing(const double *__restrict__ crossing,
                                                              const unsigned long long *__restrict__ crossing_count,
                                                              uint32_t crossing_cap, int n,
                                                              const DevView *__restrict__ views, DevOptions opt,
                                                              int rec_floats, float *__restrict__ records,
                                                              uint32_t *__restrict__ depth_keys,
                                                              uint2 *__restrict__ boxes, uint2 *__restrict__ bin_boxes,
                                                              const Conic *__restrict__ conics,
                                                              uint32_t *__restrict__ tile_counts)
{
    __shared__ double poly[2][kClipMaxVerts][3][kClipBlock];
    const unsigned long long total = min(*crossing_count, (unsigned long long)crossing_cap);
    const int l = threadIdx.x;
    for (unsigned long long j = (unsigned long long)blockIdx.x * kClipBlock + l; j < total;
         j += (unsigned long long)gridDim.x * kClipBlock) {
        const double *e = crossing + j * kCrossingDoubles;
        const uint32_t idx = (uint32_t)e[10];
        const DevView &V = views[idx / (uint32_t)n];
        const double hs = e[9];
        const double O0[4] = {-1.0, -1.0, 1.0, 1.0}, O1[4] = {-1.0, 1.0, 1.0, -1.0};
        for (int k = 0; k < 4; ++k) {
            const double z0 = hs * O0[k], z1 = hs * O1[k];
            poly[0][k][0][l] = e[3] * z0 + e[4] * z1 + e[0];
            poly[0][k][1][l] = e[5] * z0 + e[6] * z1 + e[1];
            poly[0][k][2][l] = e[7] * z0 + e[8] * z1 + e[2];
        }
        // inside half-spaces: u >= 0, u <= W, v >= 0, v <= H (z > 0)
        const double pl[4][3] = {{V.fx, 0.0, V.cx},
                                 {-V.fx, 0.0, (double)V.width - V.cx},
                                 {0.0, V.fy, V.cy},
                                 {0.0, -V.fy, (double)V.height - V.cy}};
        int m = 4, cur = 0;
        bool bounded = true;
        for (int p = 0; p < 4 && m > 0 && bounded; ++p) {
            int k = 0;
            for (int a = 0; a < m; ++a) {
                const int bi = a + 1 == m ? 0 : a + 1;
                double A[3], B[3];
                for (int c = 0; c < 3; ++c) {
                    A[c] = poly[cur][a][c][l];
                    B[c] = poly[cur][bi][c][l];
                }
                const double da = pl[p][0] * A[0] + pl[p][1] * A[1] + pl[p][2] * A[2];
                const double db = pl[p][0] * B[0] + pl[p][1] * B[1] + pl[p][2] * B[2];
                const int emit = (da >= 0.0 ? 1 : 0) + ((da >= 0.0) != (db >= 0.0) ? 1 : 0);
                if (k + emit > kClipMaxVerts) {
                    bounded = false;
                    break;
                }
                if (da >= 0.0) {
                    for (int c = 0; c < 3; ++c) poly[1 - cur][k][c][l] = A[c];
                    ++k;
                }
                if ((da >= 0.0) != (db >= 0.0)) {
                    const double t = da / (da - db);
                    for (int c = 0; c < 3; ++c) poly[1 - cur][k][c][l] = A[c] + t * (B[c] - A[c]);
                    ++k;
                }
            }
            m = k;
            cur = 1 - cur;
        }
        if (!bounded) continue;
        int px0 = 1, px1 = 0, py0 = 1, py1 = 0;
        if (m > 0) {
            double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
            for (int a = 0; a < m && bounded; ++a) {
                const double z = poly[cur][a][2][l];
                if (!(z > 0.0)) {
                    bounded = false;
                    break;
                }
                const double iz = 1.0 / z;
                const double u = V.fx * poly[cur][a][0][l] * iz + V.cx;
                const double vv = V.fy * poly[cur][a][1][l] * iz + V.cy;
                umin = fmin(umin, u);
                umax = fmax(umax, u);
                vmin = fmin(vmin, vv);
                vmax = fmax(vmax, vv);
            }
            if (!bounded) continue;
            const int Wd = V.width, Hd = V.height;
            const double fx0 = ceil(umin - 0.5), fx1 = floor(umax - 0.5);
            const double fy0 = ceil(vmin - 0.5), fy1 = floor(vmax - 0.5);
            px0 = fx0 < 0.0 ? 0 : (fx0 > Wd ? Wd : (int)fx0);
            px1 = fx1 > Wd - 1 ? Wd - 1 : (fx1 < -1.0 ? -1 : (int)fx1);
            py0 = fy0 < 0.0 ? 0 : (fy0 > Hd ? Hd : (int)fy0);
            py1 = fy1 > Hd - 1 ? Hd - 1 : (fy1 < -1.0 ? -1 : (int)fy1);
        }
        int bx0 = px0, bx1 = px1, by0 = py0, by1 = py1;
        if (px0 > px1 || py0 > py1 || !binning_clip(conics[idx], px0, px1, py0, py1, bx0, bx1, by0, by1)) {
            depth_keys[idx] = 0xffffffffu;
            tile_counts[idx] = 0u;
            boxes[idx] = make_uint2(0u, 0u);
            bin_boxes[idx] = make_uint2(0u, 0u);
            continue;
        }
        boxes[idx] = make_uint2((uint32_t)px0 | ((uint32_t)px1 << 16), (uint32_t)py0 | ((uint32_t)py1 << 16));
        bin_boxes[idx] = make_uint2((uint32_t)bx0 | ((uint32_t)bx1 << 16), (uint32_t)by0 | ((uint32_t)by1 << 16));
        tile_counts[idx] =
            (uint32_t)(((bx1 >> opt.tile_wshift) - (bx0 >> opt.tile_wshift) + 1) * ((by1 >> opt.tile_hshift) - (by0 >> opt.tile_hshift) + 1));
        records[(size_t)idx * rec_floats + 3] = __uint_as_float((uint32_t)by0 | ((uint32_t)by1 << 16));
    }
}

}  // namespace

hipError_t launch_preprocess(const rgs_gaussians &g, const DevView *views, int n_views, const DevOptions &opt,
                             float4 *records, uint32_t *depth_keys, uint2 *boxes, uint2 *bin_boxes, Conic *conics,
                             uint32_t *tile_counts, double *crossing, int64_t *crossing_count,
                             uint32_t crossing_cap, hipStream_t stream)
{
    const int n = (int)g.n;
    if (n == 0) return hipSuccess;
    const dim3 grid((n + 255) / 256), block(256);
    const int mode = opt.divergence == RGS_DIVERGENCE_GS ? kPrepGS
                     : opt.mip == 2                     ? kPrepMipExact
                     : (opt.mip == 1 || opt.mip == 3)   ? kPrepMipApprox
                                                        : kPrepRay;
#define RGS_PRE(M, D)                                                                                            \
    k_preprocess<M, D><<<grid, block, 0, stream>>>(g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, n,    \
                                                   views, n_views, opt, records, depth_keys, boxes, bin_boxes,    \
                                                   conics,                                                        \
                                                   tile_counts, crossing,                                         \
                                                   reinterpret_cast<unsigned long long *>(crossing_count), crossing_cap)
#define RGS_PRE_DEG(M)                    \
    switch (g.sh_degree) {                \
    case 0: RGS_PRE(M, 0); break;         \
    case 1: RGS_PRE(M, 1); break;         \
    case 2: RGS_PRE(M, 2); break;         \
    default: RGS_PRE(M, 3); break;        \
    }
    switch (mode) {
    case kPrepGS: RGS_PRE_DEG(kPrepGS); break;
    case kPrepMipExact: RGS_PRE_DEG(kPrepMipExact); break;
    case kPrepMipApprox: RGS_PRE_DEG(kPrepMipApprox); break;
    default: RGS_PRE_DEG(kPrepRay); break;
    }
#undef RGS_PRE_DEG
#undef RGS_PRE
    // the linearised divergence has no quad, so nothing crosses
    if (mode != kPrepGS && crossing_cap > 0)
        k_clip_crossing<<<kClipGrid, kClipBlock, 0, stream>>>(
            crossing, reinterpret_cast<const unsigned long long *>(crossing_count), crossing_cap, n, views, opt,
            record_floats(opt.mip), reinterpret_cast<float *>(records), depth_keys, boxes, bin_boxes, conics,
            tile_counts);
    return hipGetLastError();
}

}  // namespace rgs
