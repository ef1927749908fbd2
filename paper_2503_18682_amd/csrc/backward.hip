// Per-Gaussian backward: chain rule from the accumulated raster-record
// gradients to the Gaussian parameters (means, log-scales, quaternions,
// opacity logits, SH coefficients), summed over the views of the batch.
//
// The record's 2x2 map G = R_v[:, 0:2]^T A2 enters the image only through
// q = |G delta|^2 = delta^T M delta with
//     M = G^T G = A2^T (I - mu^ mu^^T) A2 = A2^T A2 - w w^T / c^2,
// where A = S^-1 R_p^T, A2 = A[:, 0:2] diag(1/fx, 1/fy), mu' = A mu and
// w = A2^T mu' (so g = w / c^2).  The compositing kernel therefore
// accumulates dL/dM, and this kernel differentiates M, g, k0 = 1/mu_z,
// ic2 = 1/c^2 and the projected centre with respect to (A, mu) without ever
// differentiating the rotation R_{mu^ <- v}.  Geometry is evaluated in double
// precision; the colour part in float32, as the forward computed it.
#include "internal.h"
#include "sh.h"

namespace rgs {
namespace {

// Chain through the MIP transform (Sec. 5, eq. 17).  With s0 the scales,
// o0 the prior opacity, ml = R_p^T mu and tau^2 = |mu|^2:
//   s_k^2 = s0_k^2 + sigma^2 tau^2,
//   log o = log o0 + log|S0| + (1/2) log c2p - log|S| - (1/2) log c2h,
//   c2p = sum_k ml_k^2 / s0_k^2,  c2h = sum_k ml_k^2 / s_k^2.
// Given dL/dlog s_k (dls) and dL/dlog o (Lo) of the rendered values, adds
// the gradients with respect to log s0 (dl), mu (dmu) and R_p (dRp).
__device__ void mip_chain(const double (&mu)[3], const double (&Rp)[9], const double (&s0)[3], const double (&s)[3],
                          double sigma2, const double (&dls)[3], double Lo, double (&dl)[3], double (&dmu)[3],
                          double (&dRp)[9])
{
    double ml[3], is0[3], is[3];
    for (int k = 0; k < 3; ++k) {
        ml[k] = Rp[k] * mu[0] + Rp[3 + k] * mu[1] + Rp[6 + k] * mu[2];
        is0[k] = 1.0 / (s0[k] * s0[k]);
        is[k] = 1.0 / (s[k] * s[k]);
    }
    double c2p = 0.0, c2h = 0.0, ml2s4 = 0.0, is_sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        c2p += ml[k] * ml[k] * is0[k];
        c2h += ml[k] * ml[k] * is[k];
        ml2s4 += ml[k] * ml[k] * is[k] * is[k];
        is_sum += is[k];
    }
    const double ic2p = 1.0 / c2p, ic2h = 1.0 / c2h;
    double tau_term = 0.0;  // dL/dlog s_k summed against dlog s_k / d(tau^2)
    for (int k = 0; k < 3; ++k) {
        const double r = s0[k] * s0[k] * is[k];  // dlog s_k / dlog s0_k
        dl[k] += dls[k] * r + Lo * (1.0 - ml[k] * ml[k] * is0[k] * ic2p - r + ml[k] * ml[k] * is[k] * r * ic2h);
        tau_term += dls[k] * is[k];
    }
    double a0[3], a1[3];
    for (int k = 0; k < 3; ++k) {
        a0[k] = ml[k] * is0[k] * ic2p - ml[k] * is[k] * ic2h;  // dlog o / d ml_k
        a1[k] = Lo * a0[k];
    }
    const double mu_coef = sigma2 * (tau_term + Lo * (ml2s4 * ic2h - is_sum));
    for (int j = 0; j < 3; ++j)
        dmu[j] += mu_coef * mu[j] + Rp[3 * j] * a1[0] + Rp[3 * j + 1] * a1[1] + Rp[3 * j + 2] * a1[2];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dRp[3 * r + k] += a1[k] * mu[r];
}

// Chain of the linearised divergence (Sec. 3.1): the record holds
// pi(mu) (gradient gc) and G with G^T G = A = Sigma_pi^-1 (gradient GA as a
// symmetric matrix), Sigma_pi = J Sigma J^T with J(mu) the pinhole Jacobian
// and Sigma = R_p S^2 R_p^T.  dL/dSigma_pi = -A GA A; dL/dSigma =
// J^T (dL/dSigma_pi) J; dL/dJ = 2 (dL/dSigma_pi) J Sigma; pi has Jacobian J.
// Adds dL/dmu, dL/dR_p and dL/dlog s.
__device__ void gs_chain(const double mu[3], const double Rp[9], const double s[3], const DevView &V,
                         const double sq[2], const double GA[2][2], double dmu[3], double dRp[9], double dls[3])
{
    const double iz = 1.0 / mu[2];
    const double J[2][3] = {{V.fx * iz, 0.0, -V.fx * mu[0] * iz * iz}, {0.0, V.fy * iz, -V.fy * mu[1] * iz * iz}};
    double M[2][3];  // J R_p S
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) M[r][c] = (J[r][0] * Rp[c] + J[r][1] * Rp[3 + c] + J[r][2] * Rp[6 + c]) * s[c];
    const double P00 = M[0][0] * M[0][0] + M[0][1] * M[0][1] + M[0][2] * M[0][2];
    const double P01 = M[0][0] * M[1][0] + M[0][1] * M[1][1] + M[0][2] * M[1][2];
    const double P11 = M[1][0] * M[1][0] + M[1][1] * M[1][1] + M[1][2] * M[1][2];
    const double idet = 1.0 / (P00 * P11 - P01 * P01);
    const double A[2][2] = {{P11 * idet, -P01 * idet}, {-P01 * idet, P00 * idet}};
    // the anchor's gradient from the record's raw q sums (its M is A, g = 0)
    const double gc[2] = {A[0][0] * sq[0] + A[0][1] * sq[1], A[1][0] * sq[0] + A[1][1] * sq[1]};
    double T[2][2], GP[2][2];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) T[r][c] = GA[r][0] * A[0][c] + GA[r][1] * A[1][c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) GP[r][c] = -(A[r][0] * T[0][c] + A[r][1] * T[1][c]);
    // Sigma = (R_p S)(R_p S)^T
    double Sig[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += Rp[3 * a + k] * Rp[3 * b + k] * s[k] * s[k];
            Sig[a][b] = acc;
        }
    double PJ[2][3];  // GP J
    for (int r = 0; r < 2; ++r)
        for (int a = 0; a < 3; ++a) PJ[r][a] = GP[r][0] * J[0][a] + GP[r][1] * J[1][a];
    double GS[3][3];  // J^T GP J
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) GS[a][b] = J[0][a] * PJ[0][b] + J[1][a] * PJ[1][b];
    double GJ[2][3];  // 2 GP J Sigma
    for (int r = 0; r < 2; ++r)
        for (int b = 0; b < 3; ++b) GJ[r][b] = 2.0 * (PJ[r][0] * Sig[0][b] + PJ[r][1] * Sig[1][b] + PJ[r][2] * Sig[2][b]);
    for (int a = 0; a < 3; ++a) dmu[a] += J[0][a] * gc[0] + J[1][a] * gc[1];
    const double iz2 = iz * iz, iz3 = iz2 * iz;
    dmu[0] += GJ[0][2] * (-V.fx * iz2);
    dmu[1] += GJ[1][2] * (-V.fy * iz2);
    dmu[2] += GJ[0][0] * (-V.fx * iz2) + GJ[0][2] * (2.0 * V.fx * mu[0] * iz3) + GJ[1][1] * (-V.fy * iz2) +
              GJ[1][2] * (2.0 * V.fy * mu[1] * iz3);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            dRp[3 * r + c] += 2.0 * (GS[r][0] * Rp[c] + GS[r][1] * Rp[3 + c] + GS[r][2] * Rp[6 + c]) * s[c] * s[c];
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) acc += Rp[3 * a + k] * GS[a][b] * Rp[3 * b + k];
        dls[k] += 2.0 * s[k] * s[k] * acc;
    }
}

// Chain of the exact MIP record (mip = 2; written by write_exact_mip_record):
// from the gradient of its values gr (kGradFloatsExactMip layout) to dL/dmu,
// dL/dR_p, dL/ds (added) and dL/do (returned).  With lam = s_max^2:
//   P0_k = R_p[0][k] / fx, P1_k = R_p[1][k] / fy,
//   Q0_k = (R_p[1][k] mu_z - mu_y R_p[2][k]) / (fx s_max),
//   Q1_k = (mu_x R_p[2][k] - R_p[0][k] mu_z) / (fy s_max),
//   rho_k = (R_p^T mu)_k / mu_z, s'^2_k = s_k^2 / lam, e = sigma^2 mu_z^2 / lam,
//   log2o = log2 o + sum_k log2 s'^2_k / 2, centre = (fx mu_x / mu_z + cx, fy mu_y / mu_z + cy).
__device__ double exact_mip_chain(const double mu[3], const double Rp[9], const double s[3], double o,
                                  const DevView &V, double sig2, const float *gr, double dmu[3], double dRp[9],
                                  double ds[3])
{
    constexpr double kLn2 = 0.69314718055994531;
    int m = 0;
    for (int k = 1; k < 3; ++k)
        if (s[k] > s[m]) m = k;
    const double smax = s[m], ilam = 1.0 / (smax * smax), iz = 1.0 / mu[2];
    const double ax = 1.0 / (V.fx * smax), ay = 1.0 / (V.fy * smax);
    const double gcx = gr[0], gcy = gr[1], ge = gr[20], glog2o = gr[21];
    double dsmax = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double gP0 = gr[2 + k], gP1 = gr[5 + k], gQ0 = gr[8 + k], gQ1 = gr[11 + k], grho = gr[14 + k];
        const double s2 = s[k] * s[k] * ilam;
        const double gs2 = gr[17 + k] + glog2o * 0.5 / (s2 * kLn2);
        const double Q0 = (Rp[3 + k] * mu[2] - mu[1] * Rp[6 + k]) * ax;
        const double Q1 = (mu[0] * Rp[6 + k] - Rp[k] * mu[2]) * ay;
        const double rho = (Rp[k] * mu[0] + Rp[3 + k] * mu[1] + Rp[6 + k] * mu[2]) * iz;
        dRp[k] += gP0 / V.fx - gQ1 * mu[2] * ay + grho * mu[0] * iz;
        dRp[3 + k] += gP1 / V.fy + gQ0 * mu[2] * ax + grho * mu[1] * iz;
        dRp[6 + k] += -gQ0 * mu[1] * ax + gQ1 * mu[0] * ay + grho * mu[2] * iz;
        dmu[0] += gQ1 * Rp[6 + k] * ay + grho * Rp[k] * iz;
        dmu[1] += -gQ0 * Rp[6 + k] * ax + grho * Rp[3 + k] * iz;
        dmu[2] += gQ0 * Rp[3 + k] * ax - gQ1 * Rp[k] * ay + grho * (Rp[6 + k] - rho) * iz;
        dsmax -= (gQ0 * Q0 + gQ1 * Q1 + gs2 * 2.0 * s2) / smax;
        ds[k] += gs2 * 2.0 * s[k] * ilam;
    }
    const double e = sig2 * mu[2] * mu[2] * ilam;
    dmu[2] += ge * 2.0 * e * iz;
    dsmax -= ge * 2.0 * e / smax;
    ds[m] += dsmax;
    dmu[0] += gcx * V.fx * iz;
    dmu[1] += gcy * V.fy * iz;
    dmu[2] -= (gcx * V.fx * mu[0] + gcy * V.fy * mu[1]) * iz * iz;
    return glog2o / (o * kLn2);
}

// Zeroes the record gradients of the kept Gaussian-views, the only ones the
// backward kernels add into or read (the depth order lists them first:
// order[0, *kept)).  One thread per float4, so each record's lines are
// written whole.
__global__ __launch_bounds__(256) void k_zero_kept_grads(const uint32_t *__restrict__ order,
                                                         const int64_t *__restrict__ kept_p, int64_t n_max,
                                                         int stride4, float4 *__restrict__ grads)
{
    // consecutive threads clear consecutive float4 of one record gradient, so
    // each record's line is written whole by one store instruction (stride4 is
    // a power of two: the entry and part are a shift and a mask)
    const int64_t kept = min(*kept_p, n_max);
    const int sh = __builtin_ctz((unsigned)stride4);
    const int64_t total = kept << sh;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i >> sh;
        grads[((size_t)order[e] << sh) + (size_t)(i & (stride4 - 1))] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Geometry and opacity (the colour part is k_colour_bwd).
// One instantiation per divergence and MIP mode (as the forward preprocess),
// so that each carries only its own chain.
enum BwdMode { kBwdRay = 0, kBwdMip = 1, kBwdMipExact = 2, kBwdGS = 3 };

template <int MODE>
__global__ __launch_bounds__(256) void k_preprocess_bwd(
    const float *__restrict__ means, const float *__restrict__ log_scales, const float *__restrict__ quats,
    const float *__restrict__ opacity_logits, int n, const DevView *__restrict__ views, int n_views,
    const uint32_t *__restrict__ tile_counts, const float *__restrict__ record_grads, DevOptions opt,
    float *__restrict__ g_means, float *__restrict__ g_log_scales, float *__restrict__ g_quats,
    float *__restrict__ g_opacity)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool any = false;
    for (int v = 0; v < n_views; ++v) any = any || tile_counts[(size_t)v * n + i] != 0;
    if (!any) return;

    const double m[3] = {means[i], means[n + i], means[2 * n + i]};
    const double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    // repeated divisors are applied as one reciprocal each (a double division
    // is a long instruction sequence; gradients need no exact rounding)
    const double iq = 1.0 / qn;
    const double w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
    double R[9];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
    const double s[3] = {exp((double)log_scales[i]), exp((double)log_scales[n + i]), exp((double)log_scales[2 * n + i])};
    const double is[3] = {1.0 / s[0], 1.0 / s[1], 1.0 / s[2]};
    const double o = 1.0 / (1.0 + exp(-(double)opacity_logits[i]));

    double dm[3] = {0, 0, 0}, dl[3] = {0, 0, 0}, dR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, da = 0.0;

    for (int v = 0; v < n_views; ++v) {
        const size_t idx = (size_t)v * n + i;
        if (tile_counts[idx] == 0) continue;
        const DevView &V = views[v];
        const float *gr = record_grads + idx * (MODE == kBwdMipExact ? kGradFloatsExactMip : kGradFloats);
        if constexpr (MODE == kBwdMipExact) {
            const double mu[3] = {V.w2c[0] * m[0] + V.w2c[1] * m[1] + V.w2c[2] * m[2] + V.w2c[3],
                                  V.w2c[4] * m[0] + V.w2c[5] * m[1] + V.w2c[6] * m[2] + V.w2c[7],
                                  V.w2c[8] * m[0] + V.w2c[9] * m[1] + V.w2c[10] * m[2] + V.w2c[11]};
            double Rp[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    Rp[3 * r + c] = V.w2c[4 * r] * R[c] + V.w2c[4 * r + 1] * R[3 + c] + V.w2c[4 * r + 2] * R[6 + c];
            double dmu[3] = {0, 0, 0}, dRp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ds[3] = {0, 0, 0};
            const double go = exact_mip_chain(mu, Rp, s, o, V, opt.mip_sigma2_px / (V.fx * V.fy), gr, dmu, dRp, ds);
            const double *W = V.w2c;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    dR[3 * r + c] += W[r] * dRp[c] + W[4 + r] * dRp[3 + c] + W[8 + r] * dRp[6 + c];
            for (int c = 0; c < 3; ++c) dm[c] += W[c] * dmu[0] + W[4 + c] * dmu[1] + W[8 + c] * dmu[2];
            for (int k = 0; k < 3; ++k) dl[k] += ds[k] * s[k];
            da += go * o * (1.0 - o);
            continue;
        }
        // the record's gradient from the raw sums of the backward compositing
        // kernel (layout at kGradFloats): the q moments are -2 dL/dM sums
        // (dM01 counts the off-diagonal twice), the dic2 sum 2 dL/d(1/c^2) in
        // the test form's units, which scale by 1 / s^2 = 2 ln 2 K per power of
        // den (dk0, dg, du0, dv0) and by 1 / s^4 for 1/c^2
        const double gM00 = -0.5 * (double)gr[2], gM01 = -(double)gr[3], gM11 = -0.5 * (double)gr[4];
        // gr[9] = sum of w dL/dw = the record opacity ov times dL/dov
        const double sqx = gr[0], sqy = gr[1], sd = gr[7], gw = gr[9];
        const double *W = V.w2c;
        const double mu[3] = {W[0] * m[0] + W[1] * m[1] + W[2] * m[2] + W[3],
                              W[4] * m[0] + W[5] * m[1] + W[6] * m[2] + W[7],
                              W[8] * m[0] + W[9] * m[1] + W[10] * m[2] + W[11]};
        double Rp[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Rp[3 * r + c] = W[4 * r] * R[c] + W[4 * r + 1] * R[3 + c] + W[4 * r + 2] * R[6 + c];
        if constexpr (MODE == kBwdGS) {
            // the record's anchor is pi(mu) and its M = G^T G is Sigma_pi^-1;
            // den, g, 1/c^2 are constants of this divergence
            const double sq[2] = {sqx, sqy};
            const double GA[2][2] = {{gM00, 0.5 * gM01}, {0.5 * gM01, gM11}};
            double dmu[3] = {0, 0, 0}, dRp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            gs_chain(mu, Rp, s, V, sq, GA, dmu, dRp, dl);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    dR[3 * r + c] += W[r] * dRp[c] + W[4 + r] * dRp[3 + c] + W[8 + r] * dRp[6 + c];
            for (int c = 0; c < 3; ++c) dm[c] += W[c] * dmu[0] + W[4 + c] * dmu[1] + W[8 + c] * dmu[2];
            da += gw * (1.0 - o);
            continue;
        }
        // rendered scales and opacity: widened by the MIP transform when it is on
        double sv[3] = {s[0], s[1], s[2]}, isv[3] = {is[0], is[1], is[2]};
        double ov = o;
        const double sig2 = MODE == kBwdMip ? opt.mip_sigma2_px / (V.fx * V.fy) : 0.0;
        if constexpr (MODE == kBwdMip) {
            const double tb2 = mu[0] * mu[0] + mu[1] * mu[1] + mu[2] * mu[2];
            double det = 1.0, deth = 1.0, c2p = 0.0, c2h = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double ml = Rp[k] * mu[0] + Rp[3 + k] * mu[1] + Rp[6 + k] * mu[2];
                const double s2 = s[k] * s[k], sh2 = s2 + sig2 * tb2;
                det *= s2;
                deth *= sh2;
                c2p += ml * ml / s2;
                c2h += ml * ml / sh2;
                sv[k] = sqrt(sh2);
                isv[k] = 1.0 / sv[k];
            }
            ov = o * sqrt(det * c2p / (deth * c2h));
        }
        double A[3][3];  // A = S^-1 R_p^T
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) A[k][j] = Rp[3 * j + k] * isv[k];
        double mw[3];
        for (int k = 0; k < 3; ++k) mw[k] = A[k][0] * mu[0] + A[k][1] * mu[1] + A[k][2] * mu[2];
        const double c2 = mw[0] * mw[0] + mw[1] * mw[1] + mw[2] * mw[2];
        const double ic2 = 1.0 / c2, ic4 = ic2 * ic2;
        const double ifx = 1.0 / V.fx, ify = 1.0 / V.fy;
        double A2[3][2];
        for (int k = 0; k < 3; ++k) {
            A2[k][0] = A[k][0] * ifx;
            A2[k][1] = A[k][1] * ify;
        }
        double wv[2];
        for (int c = 0; c < 2; ++c) wv[c] = A2[0][c] * mw[0] + A2[1][c] * mw[1] + A2[2][c] * mw[2];
        // the record's M = G^T G = A2^T A2 - w w^T / c^2 and g = w / c^2, and the
        // test form's 1 / s^2 = 2 ln 2 K with K = log2(ov / p_min)
        double Mg[3] = {-wv[0] * wv[0] * ic2, -wv[0] * wv[1] * ic2, -wv[1] * wv[1] * ic2};
        for (int k = 0; k < 3; ++k) {
            Mg[0] += A2[k][0] * A2[k][0];
            Mg[1] += A2[k][0] * A2[k][1];
            Mg[2] += A2[k][1] * A2[k][1];
        }
        // (single precision, as the record's own log2 of its opacity)
        const double is2 = 1.38629436111989061 * (double)(__log2f((float)ov) - __log2f((float)opt.p_min));
        const double ggx = is2 * gr[5], ggy = is2 * gr[6], gk0 = is2 * sd;
        const double gic2 = 0.5 * is2 * is2 * gr[8];
        const double gu0 = Mg[0] * sqx + Mg[1] * sqy - is2 * (wv[0] * ic2) * sd;
        const double gv0 = Mg[1] * sqx + Mg[2] * sqy - is2 * (wv[1] * ic2) * sd;
        // symmetric matrix gradient of M (the off-diagonal parameter appears twice)
        const double Gm[2][2] = {{gM00, 0.5 * gM01}, {0.5 * gM01, gM11}};
        double dA2[3][2], dw[2], dc2;
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 2; ++c) dA2[k][c] = 2.0 * (A2[k][0] * Gm[0][c] + A2[k][1] * Gm[1][c]);
        const double Gw[2] = {Gm[0][0] * wv[0] + Gm[0][1] * wv[1], Gm[1][0] * wv[0] + Gm[1][1] * wv[1]};
        dw[0] = (-2.0 * Gw[0] + ggx) * ic2;
        dw[1] = (-2.0 * Gw[1] + ggy) * ic2;
        dc2 = ((wv[0] * Gw[0] + wv[1] * Gw[1]) - (ggx * wv[0] + ggy * wv[1]) - gic2) * ic4;
        // w = A2^T mu'
        double dmw[3];
        for (int k = 0; k < 3; ++k) {
            dA2[k][0] += mw[k] * dw[0];
            dA2[k][1] += mw[k] * dw[1];
            dmw[k] = A2[k][0] * dw[0] + A2[k][1] * dw[1] + 2.0 * mw[k] * dc2;
        }
        // mu' = A mu, A2 = A[:, 0:2] diag(1/fx, 1/fy)
        double dA[3][3], dmu[3];
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) dA[k][j] = dmw[k] * mu[j];
        for (int k = 0; k < 3; ++k) {
            dA[k][0] += dA2[k][0] * ifx;
            dA[k][1] += dA2[k][1] * ify;
        }
        for (int j = 0; j < 3; ++j) dmu[j] = A[0][j] * dmw[0] + A[1][j] * dmw[1] + A[2][j] * dmw[2];
        // k0 = 1/mu_z, projected centre (u0, v0)
        const double iz = 1.0 / mu[2];
        dmu[2] += -gk0 * iz * iz;
        dmu[0] += gu0 * V.fx * iz;
        dmu[1] += gv0 * V.fy * iz;
        dmu[2] += -(gu0 * V.fx * mu[0] + gv0 * V.fy * mu[1]) * iz * iz;
        // A[k][j] = R_p[j][k] / s_k
        double dRp[9], dls[3];
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j) {
                dRp[3 * j + k] = dA[k][j] * isv[k];
                acc += dA[k][j] * A[k][j];
            }
            dls[k] = -acc;
        }
        // the record's opacity is ov: dL/dlog ov = go ov
        if constexpr (MODE == kBwdMip) {
            mip_chain(mu, Rp, s, sv, sig2, dls, gw, dl, dmu, dRp);
        } else {
            for (int k = 0; k < 3; ++k) dl[k] += dls[k];
        }
        // R_p = W_rot R, mu = W_rot m + t
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) dR[3 * r + c] += W[r] * dRp[c] + W[4 + r] * dRp[3 + c] + W[8 + r] * dRp[6 + c];
        for (int c = 0; c < 3; ++c) dm[c] += W[c] * dmu[0] + W[4 + c] * dmu[1] + W[8 + c] * dmu[2];
        // prior opacity: dlog o / da = 1 - o
        da += gw * (1.0 - o);
    }
    // quaternion: dR/d(w,x,y,z) of the unit quaternion, then the normalisation
    const double J[9][4] = {{0, 0, -4 * y, -4 * z},       {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
                            {2 * z, 2 * y, 2 * x, 2 * w}, {0, -4 * x, 0, -4 * z},         {-2 * x, -2 * w, 2 * z, 2 * y},
                            {-2 * y, 2 * z, -2 * w, 2 * x}, {2 * x, 2 * w, 2 * z, 2 * y}, {0, -4 * x, -4 * y, 0}};
    double dqh[4] = {0, 0, 0, 0};
    for (int e = 0; e < 9; ++e)
        for (int k = 0; k < 4; ++k) dqh[k] += dR[e] * J[e][k];
    const double qh[4] = {w, x, y, z};
    const double proj = qh[0] * dqh[0] + qh[1] * dqh[1] + qh[2] * dqh[2] + qh[3] * dqh[3];
    for (int k = 0; k < 4; ++k) g_quats[(size_t)k * n + i] += (float)((dqh[k] - qh[k] * proj) * iq);
    for (int k = 0; k < 3; ++k) {
        g_means[(size_t)k * n + i] += (float)dm[k];
        g_log_scales[(size_t)k * n + i] += (float)dl[k];
    }
    g_opacity[i] += (float)da;
}

// Colour: the SH coefficients and, through the view direction d = (m - C) /
// |m - C|, the means.  The colour is recomputed in float32 as the forward
// kernel computed it, so a channel clamped at zero there passes no gradient
// here either.
template <int DEG>
__global__ __launch_bounds__(256) void k_colour_bwd(const float *__restrict__ means, const float *__restrict__ sh,
                                                    int n, const DevView *__restrict__ views, int n_views,
                                                    const uint32_t *__restrict__ tile_counts,
                                                    const float *__restrict__ record_grads, int grad_stride,
                                                    int rgb_offset, float *__restrict__ g_means,
                                                    float *__restrict__ g_sh)
{
    constexpr int NK = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool any = false;
    for (int v = 0; v < n_views; ++v) any = any || tile_counts[(size_t)v * n + i] != 0;
    if (!any) return;
    // the gradient accumulators are read together with the coefficients, so
    // both streams of loads are in flight before any arithmetic (reading them
    // after the view loop left the final read-modify-write exposed)
    float c[NK * 3], dsh[NK * 3];
#pragma unroll
    for (int k = 0; k < NK * 3; ++k) {
        c[k] = sh[(size_t)k * n + i];
        dsh[k] = g_sh[(size_t)k * n + i];
    }
    const double m[3] = {means[i], means[n + i], means[2 * n + i]};
    double dm[3] = {0, 0, 0};
    for (int v = 0; v < n_views; ++v) {
        const size_t idx = (size_t)v * n + i;
        if (tile_counts[idx] == 0) continue;
        const DevView &V = views[v];
        const float *gr = record_grads + idx * grad_stride;
        float dir[3];
        double dist;
        view_dir(m, V.centre, dir, &dist);
        float Y[NK], col[3];
        sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
        sh_colour<DEG>(Y, c, col);
        // channels clamped at zero in the forward pass no gradient
        float gcol[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gcol[ch] = col[ch] > 0.0f ? gr[rgb_offset + ch] : 0.0f;
        float wk[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            wk[k] = 0.0f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                dsh[3 * k + ch] += Y[k] * gcol[ch];
                wk[k] += gcol[ch] * c[3 * k + ch];
            }
        }
        float ddir[3];
        sh_dir_grad<DEG>(dir[0], dir[1], dir[2], wk, ddir);
        const double pd = (double)ddir[0] * dir[0] + (double)ddir[1] * dir[1] + (double)ddir[2] * dir[2];
        const double idist = 1.0 / dist;
        for (int j = 0; j < 3; ++j) dm[j] += ((double)ddir[j] - dir[j] * pd) * idist;
    }
    for (int k = 0; k < 3; ++k) g_means[(size_t)k * n + i] += (float)dm[k];
#pragma unroll
    for (int k = 0; k < NK * 3; ++k) g_sh[(size_t)k * n + i] = dsh[k];
}

}  // namespace

hipError_t launch_zero_kept_grads(const uint32_t *order, const int64_t *kept, int64_t n_max, int grad_floats_per,
                                  float *grads, int num_cus, hipStream_t stream)
{
    if (n_max == 0) return hipSuccess;
    const int64_t want = (n_max * (grad_floats_per / 4) + 255) / 256;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cus * 16));
    k_zero_kept_grads<<<grid, 256, 0, stream>>>(order, kept, n_max, grad_floats_per / 4,
                                                reinterpret_cast<float4 *>(grads));
    return hipGetLastError();
}

hipError_t launch_preprocess_backward(const rgs_gaussians &g, const DevView *views, int n_views,
                                      const DevOptions &opt, const uint32_t *tile_counts, const float *record_grads,
                                      const rgs_gaussian_grads &gr, hipStream_t stream)
{
    const int n = (int)g.n;
    if (n == 0) return hipSuccess;
    const dim3 grid((n + 255) / 256), block(256);
    const int mode = opt.divergence == RGS_DIVERGENCE_GS ? kBwdGS : opt.mip == 2 ? kBwdMipExact : opt.mip == 1 ? kBwdMip : kBwdRay;
#define RGS_PBWD(M)                                                                                             \
    k_preprocess_bwd<M><<<grid, block, 0, stream>>>(g.means, g.log_scales, g.quats, g.opacity_logits, n, views, \
                                                    n_views, tile_counts, record_grads, opt, gr.means,          \
                                                    gr.log_scales, gr.quats, gr.opacity_logits)
    switch (mode) {
    case kBwdGS: RGS_PBWD(kBwdGS); break;
    case kBwdMipExact: RGS_PBWD(kBwdMipExact); break;
    case kBwdMip: RGS_PBWD(kBwdMip); break;
    default: RGS_PBWD(kBwdRay); break;
    }
#undef RGS_PBWD
    // after k_preprocess_bwd on the same stream: both add into gr.means
#define RGS_BWD(D)                                                                                                  \
    k_colour_bwd<D><<<grid, block, 0, stream>>>(g.means, g.sh, n, views, n_views, tile_counts, record_grads,        \
                                                grad_floats(opt.mip), opt.mip == 2 ? 22 : 10, gr.means, gr.sh)
    switch (g.sh_degree) {
    case 0: RGS_BWD(0); break;
    case 1: RGS_BWD(1); break;
    case 2: RGS_BWD(2); break;
    default: RGS_BWD(3); break;
    }
#undef RGS_BWD
    return hipGetLastError();
}

}  // namespace rgs
