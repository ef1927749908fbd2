/*
 * raygs_oracle.c -- plain, slow FP64 CPU oracle for ray-based Gaussian
 * splatting ("Hardware-Rasterized Ray-Based Gaussian Splatting", CVPR 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or constant table with the HIP renderer and must never be used as a
 * fallback for it.
 *
 * What it computes, in the paper's order and notation (every quantity in
 * double precision; float32 inputs are widened exactly):
 *   per view, per Gaussian
 *     mu = W m + t (camera frame, Sec. 3 "Scene representation"),
 *     Sigma = R_p S^2 R_p^T with R_p = W R(q / |q|), S = diag(exp(l)),
 *     o = sigmoid(a),
 *     optional MIP widening and opacity modulation (Sec. 5, eq. 17),
 *     or, for the exact MIP density of Sec. 5 / App. A.5, a widened Gaussian
 *     that bounds its support (see mip_exact_bound),
 *     kappa = -2 log(p_min / o) (eq. 3), skipped when kappa <= 0,
 *     c^2 = mu^T Sigma^-1 mu (eq. 6), skipped when c^2 <= kappa,
 *     the 3D quad V_ray = T_ray H(Z_ray) (Sec. 4.1, eqs. 12-15, App. A.1-A.3),
 *     its pixel bounding box and tile rectangle, the depth key;
 *   per pixel
 *     every Gaussian whose box holds the pixel centre, in ascending
 *     (depth, index) order, with D_ray from its definition (eq. 5),
 *     omega = o exp(-D/2) (eq. 2), composited front to back (eq. 1);
 *     with exact MIP, omega is the per-ray MIP weight (orc_mip_exact_weight).
 *   backward (not in the paper): the exact adjoint of the above, with the
 *     derivative of D_ray taken by the envelope theorem at tau (Prop. A.1).
 *
 * Readings of points the paper leaves open (shared with the GPU path through
 * the documented options, not through code):
 *   p_min = 1/255; alpha = min(omega, alpha_max); a Gaussian contributes iff
 *   omega >= p_min; compositing stops before a Gaussian whose contribution
 *   would take the transmittance below t_eps; rays with tau <= 0 get no
 *   contribution; near-plane culling of centres with mu_z <= near_z; a quad
 *   with a vertex at z <= 0 is clipped to the side planes of the view
 *   frustum and its box is that of the clipped part; pixel centres sit at +1/2;
 *   colour = max(0, SH(view direction) + 0.5); depth key = bits of
 *   float32(mu_z), ties broken by Gaussian index.
 *
 * The linearised divergence of Sec. 3.1 (divergence = 1) replaces D_ray by
 * D_gs(x) = (pi(x) - pi(mu))^T Sigma_pi^-1 (pi(x) - pi(mu)), Sigma_pi =
 * J Sigma J^T with J the Jacobian of the pinhole projection at mu (pixel
 * units), no low-pass term; its support D_gs <= kappa is an ellipse in the
 * image, bounded by its axis-aligned box; no MIP; the near-plane and kappa
 * culls apply, the camera-inside skip does not.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ types */
typedef struct {
    double w2c[12]; /* row-major [W | t], world -> camera, OpenCV axes */
    double fx, fy, cx, cy;
    int32_t width, height;
} orc_camera;

typedef struct {
    double p_min, alpha_max, t_eps, near_z;
    int32_t mip;
    double mip_sigma2_px;
    double background[3];
    int32_t tile_w, tile_h;
    int32_t divergence; /* 0 = D_ray (eq. 5), 1 = D_gs of the linearised projection (Sec. 3.1) */
} orc_options;

typedef struct {
    const double *means, *log_scales, *quats, *opacity_logits, *sh;
    int64_t n;
    int32_t sh_degree;
} orc_scene;

enum {
    ORC_VISIBLE = 0,
    ORC_CULL_INVALID = 1,
    ORC_CULL_NEAR = 2,
    ORC_CULL_KAPPA = 3,
    ORC_CULL_INSIDE = 4,
    ORC_CULL_OFFSCREEN = 5,
    ORC_CULL_NOTILE = 6,
    ORC_CULL_NOBIN = 7   /* no pixel centre of the box lies in the support's bounding box */
};

enum { /* hazard bits: a decision taken within rounding distance */
    ORC_HZ_KEY = 1,
    ORC_HZ_RECT = 2,
    ORC_HZ_EIGEN = 4,
    ORC_HZ_CULL = 8,
    ORC_HZ_FRONT = 16
};

typedef struct {
    int32_t cull;     /* ORC_VISIBLE or the reason it was dropped */
    int32_t hazard;   /* ORC_HZ_* bits */
    double mu[3];     /* centre, camera frame */
    double Rp[9];     /* rotation, camera frame, row-major */
    double s[3];      /* scales (after MIP widening) */
    double o;         /* opacity (after MIP modulation) */
    double kappa, c2;
    double mu_w[3];   /* whitened centre S^-1 R_p^T mu */
    double b;         /* sqrt(1 - kappa / c^2) */
    double Rv[9];     /* R_{mu^ <- v}, row-major */
    double U[4];      /* U_ray = (u0, u1) as columns, row-major 2x2 */
    double quad[12];  /* 4 vertices x (x, y, z), camera frame */
    double bbox[4];   /* umin, umax, vmin, vmax of the projected quad */
    double ebox[4];   /* umin, umax, vmin, vmax of the support ellipse (infinite when unbounded) */
    int32_t all_front;
    int32_t px0, px1, py0, py1; /* pixel box: pixel centres inside bbox (inclusive) */
    int32_t bx0, bx1, by0, by1; /* binning box: pixels of the pixel box with centres inside ebox */
    int32_t tx0, tx1, ty0, ty1; /* tiles of the binning box (inclusive) */
    uint32_t depth_key;
    int32_t pad;
    double rgb[3], rgb_raw[3];
    double dir[3];    /* unit view direction used for the colour */
    double dist;      /* |m - camera centre| */
    double cq[6];     /* support conic in pixel coordinates: A00, A01, A11, b0, b1, c */
    int32_t bounded;  /* the conic is an ellipse (A positive definite) */
    int32_t listed;   /* tiles listed for this Gaussian */
    double s0[3];     /* exact MIP: scales of the Gaussian itself (s holds the bound's) */
    double sig2;      /* exact MIP: sigma^2 at the principal point, per unit distance */
    int32_t exact;    /* exact MIP weight per ray */
    int32_t whole;    /* exact MIP without a bounding Gaussian: the whole view */
    int32_t gs;       /* D_gs: the pixel-space Gaussian below */
    int32_t pad2;
    double gs_A[3];   /* Sigma_pi^-1 (A00, A01, A11), pixel units */
    double gs_c[2];   /* pi(mu), pixels */
} orc_splat;

/* --------------------------------------------------------- small helpers */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* y = M x for a row-major 3x3 M */
static void mat3_vec(const double *M, const double *x, double *y)
{
    for (int r = 0; r < 3; ++r) y[r] = M[3 * r] * x[0] + M[3 * r + 1] * x[1] + M[3 * r + 2] * x[2];
}

/* y = M^T x */
static void mat3t_vec(const double *M, const double *x, double *y)
{
    for (int c = 0; c < 3; ++c) y[c] = M[c] * x[0] + M[3 + c] * x[1] + M[6 + c] * x[2];
}

/* C = A B, row-major 3x3 */
static void mat3_mul(const double *A, const double *B, double *C)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void quat_to_rot(const double *q, double *R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------ real spherical harmonics
 * Orthonormal real SH up to degree 3, index k = l^2 + l + m, with the sign
 * convention common in Gaussian-splatting colour models (Condon-Shortley
 * phase on the odd-m terms).  Constants are the closed forms of the
 * normalisation factors. */
void orc_sh_basis(int degree, const double *d, double *Y, double *dY /* [16][3] or NULL */)
{
    const double PI = 3.14159265358979323846;
    const double c0 = 0.5 / sqrt(PI);
    const double c1 = 0.5 * sqrt(3.0 / PI);
    const double c2a = 0.5 * sqrt(15.0 / PI);
    const double c2b = 0.25 * sqrt(5.0 / PI);
    const double c2c = 0.25 * sqrt(15.0 / PI);
    const double c3a = -0.25 * sqrt(35.0 / (2.0 * PI));
    const double c3b = 0.5 * sqrt(105.0 / PI);
    const double c3c = -0.25 * sqrt(21.0 / (2.0 * PI));
    const double c3d = 0.25 * sqrt(7.0 / PI);
    const double c3e = 0.25 * sqrt(105.0 / PI);
    double x = d[0], y = d[1], z = d[2];
    double g[16][3];
    memset(g, 0, sizeof g);
    Y[0] = c0;
    if (degree >= 1) {
        Y[1] = -c1 * y; g[1][1] = -c1;
        Y[2] = c1 * z;  g[2][2] = c1;
        Y[3] = -c1 * x; g[3][0] = -c1;
    }
    if (degree >= 2) {
        Y[4] = c2a * x * y;                     g[4][0] = c2a * y; g[4][1] = c2a * x;
        Y[5] = -c2a * y * z;                    g[5][1] = -c2a * z; g[5][2] = -c2a * y;
        Y[6] = c2b * (2 * z * z - x * x - y * y); g[6][0] = -2 * c2b * x; g[6][1] = -2 * c2b * y; g[6][2] = 4 * c2b * z;
        Y[7] = -c2a * x * z;                    g[7][0] = -c2a * z; g[7][2] = -c2a * x;
        Y[8] = c2c * (x * x - y * y);           g[8][0] = 2 * c2c * x; g[8][1] = -2 * c2c * y;
    }
    if (degree >= 3) {
        Y[9] = c3a * y * (3 * x * x - y * y);
        g[9][0] = 6 * c3a * x * y; g[9][1] = c3a * (3 * x * x - 3 * y * y);
        Y[10] = c3b * x * y * z;
        g[10][0] = c3b * y * z; g[10][1] = c3b * x * z; g[10][2] = c3b * x * y;
        Y[11] = c3c * y * (4 * z * z - x * x - y * y);
        g[11][0] = -2 * c3c * x * y; g[11][1] = c3c * (4 * z * z - x * x - 3 * y * y); g[11][2] = 8 * c3c * y * z;
        Y[12] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
        g[12][0] = -6 * c3d * x * z; g[12][1] = -6 * c3d * y * z; g[12][2] = c3d * (6 * z * z - 3 * x * x - 3 * y * y);
        Y[13] = c3c * x * (4 * z * z - x * x - y * y);
        g[13][0] = c3c * (4 * z * z - 3 * x * x - y * y); g[13][1] = -2 * c3c * x * y; g[13][2] = 8 * c3c * x * z;
        Y[14] = c3e * z * (x * x - y * y);
        g[14][0] = 2 * c3e * x * z; g[14][1] = -2 * c3e * y * z; g[14][2] = c3e * (x * x - y * y);
        Y[15] = c3a * x * (x * x - 3 * y * y);
        g[15][0] = c3a * (3 * x * x - 3 * y * y); g[15][1] = -6 * c3a * x * y;
    }
    if (dY) {
        int nk = (degree + 1) * (degree + 1);
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < 3; ++j) dY[3 * k + j] = g[k][j];
    }
}

/* ----------------------------------------------------- ray divergence
 * D_ray(x; mu, Sigma) of eq. (5): tau = x^T Sigma^-1 mu / x^T Sigma^-1 x and
 * D = (tau x - mu)^T Sigma^-1 (tau x - mu), evaluated in whitened
 * coordinates (Sigma^-1 = A^T A with A = S^-1 R_p^T).  Returns D; *tau_out
 * receives tau and e_out (if not NULL) receives tau x - mu. */
double orc_divergence(const double *mu, const double *Rp, const double *s, const double *x, double *tau_out,
                      double *e_out)
{
    double xl[3], ml[3], xw[3], mw[3];
    mat3t_vec(Rp, x, xl);
    mat3t_vec(Rp, mu, ml);
    for (int k = 0; k < 3; ++k) {
        xw[k] = xl[k] / s[k];
        mw[k] = ml[k] / s[k];
    }
    double tau = dot3(xw, mw) / dot3(xw, xw);
    double D = 0.0;
    for (int k = 0; k < 3; ++k) {
        double e = tau * xw[k] - mw[k];
        D += e * e;
    }
    if (tau_out) *tau_out = tau;
    if (e_out)
        for (int k = 0; k < 3; ++k) e_out[k] = tau * x[k] - mu[k];
    return D;
}

/* Exact MIP weight of one ray (Sec. 5 and its derivation in App. A.5).
 * xbar = (u, v, 1) is the ray through a pixel centre in normalised camera
 * coordinates and x = xbar / |xbar| the unit ray.  With tau(x) the peak of the
 * Gaussian's own density along x (eq. 5) and sigma_x^2 the area that one pixel
 * subtends at unit distance along x (sigma^2 cos^3 theta, cos theta = 1/|xbar|,
 * sigma^2 its value at the principal point):
 *   Sigma^_x = Sigma + sigma_x^2 tau(x)^2 I   (the same rotation, variances
 *              s_k^2 + sigma_x^2 tau^2),
 *   omega = o m(x) exp(-D_ray(x; mu, Sigma^_x) / 2),
 *   m(x)^2 = |Sigma| x^T Sigma^-1 x / (|Sigma^_x| x^T Sigma^_x^-1 x).
 * m(x) is the ratio of the ray density's normalising factor with and without
 * the widening (both written through the determinant identity of App. A.5), so
 * it is 1 when sigma = 0 and equals the modulation of eq. (17) on the ray
 * through mu.  *tau_h receives the peak of the widened density along x; the
 * ray gets no contribution unless it is positive. */
double orc_mip_exact_weight(const double *mu, const double *Rp, const double *s0, double o, double sig2,
                            const double *xbar, double *tau_h)
{
    /* D_ray, the sign of the peak and the modulation do not depend on the
     * length of the ray vector; tau of the unit ray is |xbar| tau(xbar) */
    double nx = sqrt(dot3(xbar, xbar));
    double tau;
    orc_divergence(mu, Rp, s0, xbar, &tau, NULL);
    tau *= nx;
    double sx2 = sig2 / (nx * nx * nx);
    double a = sx2 * tau * tau;
    double sh[3], det = 1.0, deth = 1.0, xp = 0.0, xh = 0.0, xl[3];
    mat3t_vec(Rp, xbar, xl);
    for (int k = 0; k < 3; ++k) {
        double s2 = s0[k] * s0[k];
        sh[k] = sqrt(s2 + a);
        det *= s2;
        deth *= s2 + a;
        xp += xl[k] * xl[k] / s2;
        xh += xl[k] * xl[k] / (s2 + a);
    }
    double D = orc_divergence(mu, Rp, sh, xbar, tau_h, NULL);
    return o * sqrt(det * xp / (deth * xh)) * exp(-0.5 * D);
}

/* Bound of the exact MIP support.  A ray contributes only if
 * D_ray(x; mu, Sigma^_x) <= kappa (m <= 1, since det(F^T Sigma^_x F) >=
 * det(F^T Sigma F) on the tangent plane of App. A.5).  For such a ray, with
 * e = mu - tau^ x (tau^ the peak of the widened density), |e|^2 <= kappa
 * (s_max^2 + a) and the plain peak differs from tau^ by at most
 * |e| s_max / s_min, so |tau| <= |mu| + sqrt(kappa) (s_max + sigma |tau|)
 * (1 + rho), rho = s_max / s_min.  With beta = sqrt(kappa) sigma (1 + rho) < 1
 * this gives |tau| <= tau_max = (|mu| + sqrt(kappa) s_max (1 + rho)) / (1 - beta),
 * hence sigma_x^2 tau^2 <= a_max = sigma^2 tau_max^2, and D_ray decreases as
 * the covariance grows: the support lies inside the plain support (opacity o)
 * of the Gaussian widened by a_max.  Returns a_max, or -1 when beta >= 1 (no
 * bound: the whole view is listed; so it is when the bound holds the camera). */
static double mip_exact_bound(const double *mu, const double *s, double kappa, double sig2)
{
    double smax = fmax(s[0], fmax(s[1], s[2])), smin = fmin(s[0], fmin(s[1], s[2]));
    double rho = smax / smin;
    double beta = sqrt(kappa * sig2) * (1.0 + rho);
    if (!(beta < 1.0)) return -1.0;
    double tmax = (sqrt(dot3(mu, mu)) + sqrt(kappa) * smax * (1.0 + rho)) / (1.0 - beta);
    return sig2 * tmax * tmax;
}

/* R_{x,y} = 2 (x+y)(x+y)^T / |x+y|^2 - I (App. A.1) */
static void rot_align(const double *x, const double *y, double *R)
{
    double a[3] = {x[0] + y[0], x[1] + y[1], x[2] + y[2]};
    double n2 = dot3(a, a);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R[3 * r + c] = 2.0 * a[r] * a[c] / n2 - (r == c ? 1.0 : 0.0);
}

/* R_{mu^ <- v}: v = (0,0,1); R_{mu^,v} if mu^.v >= 0, else R_{mu^,-v} P with
 * P = diag(-1, 1, -1) (App. A.1). */
void orc_rot_mu_v(const double *muh, double *R)
{
    const double v[3] = {0.0, 0.0, 1.0};
    const double mv[3] = {0.0, 0.0, -1.0};
    if (muh[2] >= 0.0) {
        rot_align(muh, v, R);
    } else {
        double Rm[9];
        rot_align(muh, mv, Rm);
        /* right-multiply by P: negate columns 0 and 2 */
        for (int r = 0; r < 3; ++r) {
            R[3 * r + 0] = -Rm[3 * r + 0];
            R[3 * r + 1] = Rm[3 * r + 1];
            R[3 * r + 2] = -Rm[3 * r + 2];
        }
    }
}

static int near_integer(double v, double rel)
{
    double r = nearbyint(v);
    return fabs(v - r) <= rel * fmax(1.0, fabs(v));
}

/* Is the float32 rounding of z decided by rounding noise of size ~tol?  An
 * exact tie (z exactly on a midpoint) arises only when z was computed without
 * any rounding, which every implementation then reproduces, so it is not a
 * hazard. */
static int depth_key_hazard(double z, double tol)
{
    float f = (float)z;
    float lo = nextafterf(f, 0.0f), hi = nextafterf(f, INFINITY);
    double mlo = 0.5 * ((double)f + (double)lo), mhi = 0.5 * ((double)f + (double)hi);
    double dlo = fabs(z - mlo), dhi = fabs(z - mhi);
    return (dlo > 0.0 && dlo <= tol) || (dhi > 0.0 && dhi <= tol);
}

/* ------------------------------------------------------ tile listing
 * The pixels p whose ray x(p) = ((p_x - c_x)/f_x, (p_y - c_y)/f_y, 1) meets the
 * support satisfy D <= kappa, i.e. (c^2 - kappa) x^T Sigma^-1 x <= (x^T Sigma^-1 mu)^2
 * (eqs. 3, 5), a conic [p;1]^T C [p;1] <= 0 with
 * C = K^-T ((c^2 - kappa) Sigma^-1 - Sigma^-1 mu mu^T Sigma^-1) K^-1.  When its
 * 2x2 block is positive definite the region is one ellipse around pi(mu).  A
 * tile is listed when the rectangle spanned by its pixel centres inside the
 * Gaussian's pixel box meets that ellipse (every tile of the box when the
 * region is unbounded): every pixel centre of the support then lies in a
 * listed tile (Sec. 4.1 bounds the support; this only drops tiles of the
 * box that no part of it reaches). */
static void support_conic(orc_splat *sp, const orc_camera *cam)
{
    double Sinv[9], tmp[9], Lam[9] = {0};
    for (int k = 0; k < 3; ++k) Lam[4 * k] = 1.0 / (sp->s[k] * sp->s[k]);
    mat3_mul(sp->Rp, Lam, tmp);
    double RpT[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) RpT[3 * r + c] = sp->Rp[3 * c + r];
    mat3_mul(tmp, RpT, Sinv);
    double Sm[3];
    mat3_vec(Sinv, sp->mu, Sm);
    double N[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) N[3 * r + c] = (sp->c2 - sp->kappa) * Sinv[3 * r + c] - Sm[r] * Sm[c];
    const double Ki[9] = {1.0 / cam->fx, 0.0, -cam->cx / cam->fx, 0.0, 1.0 / cam->fy, -cam->cy / cam->fy, 0, 0, 1};
    double KiT[9], NK[9], C[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) KiT[3 * r + c] = Ki[3 * c + r];
    mat3_mul(N, Ki, NK);
    mat3_mul(KiT, NK, C);
    sp->cq[0] = C[0]; sp->cq[1] = 0.5 * (C[1] + C[3]); sp->cq[2] = C[4];
    sp->cq[3] = 0.5 * (C[2] + C[6]); sp->cq[4] = 0.5 * (C[5] + C[7]); sp->cq[5] = C[8];
    double det = sp->cq[0] * sp->cq[2] - sp->cq[1] * sp->cq[1];
    sp->bounded = sp->cq[0] > 0.0 && det > 0.0;
    if (fabs(det) <= 1e-9 * (fabs(sp->cq[0] * sp->cq[2]) + sp->cq[1] * sp->cq[1])) sp->hazard |= ORC_HZ_RECT;
}

static double conic_at(const double *q, double x, double y)
{
    return q[0] * x * x + 2.0 * q[1] * x * y + q[2] * y * y + 2.0 * (q[3] * x + q[4] * y) + q[5];
}

/* minimum of the conic over the rectangle of pixel centres [x0, x1] x [y0, y1] */
static double conic_rect_min(const double *q, int x0, int x1, int y0, int y1)
{
    double xa = x0 + 0.5, xb = x1 + 0.5, ya = y0 + 0.5, yb = y1 + 0.5;
    double det = q[0] * q[2] - q[1] * q[1];
    double px = (q[1] * q[4] - q[2] * q[3]) / det, py = (q[1] * q[3] - q[0] * q[4]) / det;
    if (px >= xa && px <= xb && py >= ya && py <= yb) return conic_at(q, px, py);
    double best = INFINITY;
    double xe[2] = {xa, xb}, ye[2] = {ya, yb};
    for (int e = 0; e < 2; ++e) {
        double y = -(q[1] * xe[e] + q[4]) / q[2];
        y = y < ya ? ya : (y > yb ? yb : y);
        best = fmin(best, conic_at(q, xe[e], y));
        double x = -(q[1] * ye[e] + q[3]) / q[0];
        x = x < xa ? xa : (x > xb ? xb : x);
        best = fmin(best, conic_at(q, x, ye[e]));
    }
    return best;
}

/* Is tile (tx, ty) listed for splat sp?  Flags a hazard when the decision is
 * within rounding of the boundary. */
static int tile_listed(orc_splat *sp, const orc_options *opt, int tx, int ty)
{
    int TW = opt->tile_w, TH = opt->tile_h;
    int cx0 = tx * TW > sp->bx0 ? tx * TW : sp->bx0;
    int cx1 = tx * TW + TW - 1 < sp->bx1 ? tx * TW + TW - 1 : sp->bx1;
    int cy0 = ty * TH > sp->by0 ? ty * TH : sp->by0;
    int cy1 = ty * TH + TH - 1 < sp->by1 ? ty * TH + TH - 1 : sp->by1;
    if (cx0 > cx1 || cy0 > cy1) return 0;
    if (!sp->bounded) return 1;
    /* scale: |conic| at the projected centre = kappa c^2 / mu_z^2 (kappa for D_gs) */
    double scale = sp->gs ? sp->kappa : sp->kappa * sp->c2 / (sp->mu[2] * sp->mu[2]);
    double m = conic_rect_min(sp->cq, cx0, cx1, cy0, cy1);
    if (fabs(m) <= 1e-9 * scale) sp->hazard |= ORC_HZ_RECT;
    return m <= 0.0;
}

/* Pixel centres inside the bounding box [umin, umax] x [vmin, vmax] (pixel x
 * covers centre x + 1/2), clipped to the view. */
static void box_to_pixels(orc_splat *sp, const orc_camera *cam, double umin, double umax, double vmin, double vmax)
{
    int W_ = cam->width, H_ = cam->height;
    sp->bbox[0] = umin; sp->bbox[1] = umax; sp->bbox[2] = vmin; sp->bbox[3] = vmax;
    double fx0 = ceil(umin - 0.5), fx1 = floor(umax - 0.5);
    double fy0 = ceil(vmin - 0.5), fy1 = floor(vmax - 0.5);
    if (near_integer(umin - 0.5, 1e-9) || near_integer(umax - 0.5, 1e-9) || near_integer(vmin - 0.5, 1e-9) ||
        near_integer(vmax - 0.5, 1e-9))
        sp->hazard |= ORC_HZ_RECT;
    sp->px0 = fx0 < 0.0 ? 0 : (fx0 > W_ ? W_ : (int)fx0);
    sp->px1 = fx1 > W_ - 1 ? W_ - 1 : (fx1 < -1.0 ? -1 : (int)fx1);
    sp->py0 = fy0 < 0.0 ? 0 : (fy0 > H_ ? H_ : (int)fy0);
    sp->py1 = fy1 > H_ - 1 ? H_ - 1 : (fy1 < -1.0 ? -1 : (int)fy1);
}

/* Binning box (tighter binning than the quad's box; the pixel box stays the
 * set of pixels evaluated): the pixels of the pixel box whose centres lie in
 * the bounding box of the support ellipse when the support conic is bounded,
 * else the pixel box itself.  No pixel centre outside it can hold support,
 * so no tile outside it can be listed.  The ellipse is
 * (x - c)^T A (x - c) <= r2 with c = -A^-1 b and r2 = -Q(c); its half widths
 * are sqrt(r2 (A^-1)_00) and sqrt(r2 (A^-1)_11).  Sets the tile range of the
 * box; returns 0 (culled, ORC_CULL_NOBIN) when it holds no pixel. */
static int binning_box(orc_splat *sp, const orc_options *opt)
{
    sp->bx0 = sp->px0; sp->bx1 = sp->px1; sp->by0 = sp->py0; sp->by1 = sp->py1;
    sp->ebox[0] = -INFINITY; sp->ebox[1] = INFINITY; sp->ebox[2] = -INFINITY; sp->ebox[3] = INFINITY;
    if (sp->bounded && !sp->gs) {
        const double *q = sp->cq;
        const double det = q[0] * q[2] - q[1] * q[1];
        const double cx = (q[1] * q[4] - q[2] * q[3]) / det, cy = (q[1] * q[3] - q[0] * q[4]) / det;
        const double r2 = -conic_at(q, cx, cy);
        const double hx = sqrt(r2 * q[2] / det), hy = sqrt(r2 * q[0] / det);
        sp->ebox[0] = cx - hx; sp->ebox[1] = cx + hx; sp->ebox[2] = cy - hy; sp->ebox[3] = cy + hy;
        const double fx0 = ceil(sp->ebox[0] - 0.5), fx1 = floor(sp->ebox[1] - 0.5);
        const double fy0 = ceil(sp->ebox[2] - 0.5), fy1 = floor(sp->ebox[3] - 0.5);
        int hz = 0;
        for (int k = 0; k < 4; ++k) hz |= near_integer(sp->ebox[k] - 0.5, 1e-9);
        if (hz) sp->hazard |= ORC_HZ_RECT;
        if (fx0 > sp->bx0) sp->bx0 = fx0 > sp->px1 + 1 ? sp->px1 + 1 : (int)fx0;
        if (fx1 < sp->bx1) sp->bx1 = fx1 < sp->px0 - 1 ? sp->px0 - 1 : (int)fx1;
        if (fy0 > sp->by0) sp->by0 = fy0 > sp->py1 + 1 ? sp->py1 + 1 : (int)fy0;
        if (fy1 < sp->by1) sp->by1 = fy1 < sp->py0 - 1 ? sp->py0 - 1 : (int)fy1;
        /* an edge within rounding can decide whether the box is empty */
        if (hz && (sp->bx1 - sp->bx0 <= 0 || sp->by1 - sp->by0 <= 0)) sp->hazard |= ORC_HZ_CULL;
    }
    if (sp->bx0 > sp->bx1 || sp->by0 > sp->by1) {
        sp->cull = ORC_CULL_NOBIN;
        return 0;
    }
    sp->tx0 = sp->bx0 / opt->tile_w; sp->tx1 = sp->bx1 / opt->tile_w;
    sp->ty0 = sp->by0 / opt->tile_h; sp->ty1 = sp->by1 / opt->tile_h;
    return 1;
}

/* The part of a quad (4 corners in order, camera frame) that can project into
 * the view: the quad clipped, Sutherland-Hodgman, against the four side
 * planes of the view frustum, which pass through the camera centre and hold
 * the image borders (inside all four, z >= 0).  Returns 1 with the bounding
 * box (umin, umax, vmin, vmax) of the projected clipped polygon, 0 when no
 * part of the quad is inside, -1 when a clipped vertex has z <= 0 (only the
 * camera centre itself can) or, from rounding alone, the polygon would
 * outgrow its buffers (a convex quad gains at most one vertex per plane). */
#define ORC_CLIP_MAX 32
static int clip_quad_to_view(const double *quad, const orc_camera *cam, double *box)
{
    double P[ORC_CLIP_MAX][3], Q[ORC_CLIP_MAX][3];
    int n = 4;
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 3; ++c) P[k][c] = quad[3 * k + c];
    const double planes[4][3] = {{cam->fx, 0.0, cam->cx},
                                 {-cam->fx, 0.0, cam->width - cam->cx},
                                 {0.0, cam->fy, cam->cy},
                                 {0.0, -cam->fy, cam->height - cam->cy}};
    for (int p = 0; p < 4; ++p) {
        int m = 0;
        for (int i = 0; i < n; ++i) {
            const double *A = P[i], *B = P[(i + 1) % n];
            double da = dot3(planes[p], A), db = dot3(planes[p], B);
            if (m + 2 > ORC_CLIP_MAX) return -1;
            if (da >= 0.0) memcpy(Q[m++], A, sizeof(double) * 3);
            if ((da >= 0.0) != (db >= 0.0)) {
                double t = da / (da - db);
                for (int c = 0; c < 3; ++c) Q[m][c] = A[c] + t * (B[c] - A[c]);
                ++m;
            }
        }
        n = m;
        if (n == 0) return 0;
        memcpy(P, Q, sizeof(double) * 3 * n);
    }
    box[0] = INFINITY; box[1] = -INFINITY; box[2] = INFINITY; box[3] = -INFINITY;
    for (int i = 0; i < n; ++i) {
        if (!(P[i][2] > 0.0)) return -1;
        double u = cam->fx * P[i][0] / P[i][2] + cam->cx, v = cam->fy * P[i][1] / P[i][2] + cam->cy;
        box[0] = fmin(box[0], u); box[1] = fmax(box[1], u);
        box[2] = fmin(box[2], v); box[3] = fmax(box[3], v);
    }
    return 1;
}

/* ------------------------------------------------------ per-Gaussian stage */
static void preprocess_one(const orc_scene *sc, int64_t i, const orc_camera *cam, const orc_options *opt,
                           orc_splat *sp)
{
    const int64_t n = sc->n;
    memset(sp, 0, sizeof *sp);
    sp->cull = ORC_CULL_INVALID;
    const double *W = cam->w2c;
    double Wr[9] = {W[0], W[1], W[2], W[4], W[5], W[6], W[8], W[9], W[10]};
    double t[3] = {W[3], W[7], W[11]};

    double m[3], l[3], q[4], a = sc->opacity_logits[i];
    for (int k = 0; k < 3; ++k) {
        m[k] = sc->means[k * n + i];
        l[k] = sc->log_scales[k * n + i];
    }
    for (int k = 0; k < 4; ++k) q[k] = sc->quats[k * n + i];
    int nk = (sc->sh_degree + 1) * (sc->sh_degree + 1);
    int finite = isfinite(a);
    for (int k = 0; k < 3; ++k) finite = finite && isfinite(m[k]) && isfinite(l[k]);
    for (int k = 0; k < 4; ++k) finite = finite && isfinite(q[k]);
    for (int k = 0; k < nk * 3; ++k) finite = finite && isfinite(sc->sh[(int64_t)k * n + i]);
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!finite || !(qn > 0.0)) return;

    /* camera-frame centre (Sec. 3 assumes centre and covariance in the camera frame) */
    double mu[3] = {Wr[0] * m[0] + Wr[1] * m[1] + Wr[2] * m[2] + t[0],
                    Wr[3] * m[0] + Wr[4] * m[1] + Wr[5] * m[2] + t[1],
                    Wr[6] * m[0] + Wr[7] * m[1] + Wr[8] * m[2] + t[2]};
    memcpy(sp->mu, mu, sizeof mu);
    sp->depth_key = 0;
    {
        float fz = (float)mu[2];
        memcpy(&sp->depth_key, &fz, 4);
    }
    if (depth_key_hazard(mu[2], 1e-14 * (fabs(Wr[6] * m[0]) + fabs(Wr[7] * m[1]) + fabs(Wr[8] * m[2]) + fabs(t[2]))))
        sp->hazard |= ORC_HZ_KEY;
    if (fabs(mu[2] - opt->near_z) <= 1e-12 * fmax(1.0, fabs(mu[2]))) sp->hazard |= ORC_HZ_CULL;
    if (!(mu[2] > opt->near_z)) {
        sp->cull = ORC_CULL_NEAR;
        return;
    }

    /* Sigma = R_p S^2 R_p^T with R_p = W R(q^) (Sec. 3) */
    double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double R[9];
    quat_to_rot(qh, R);
    mat3_mul(Wr, R, sp->Rp);
    double s[3] = {exp(l[0]), exp(l[1]), exp(l[2])};
    double o = 1.0 / (1.0 + exp(-a));

    if (opt->divergence == 1) {
        /* Sec. 3.1: the 2D Gaussian of the projection linearised at mu */
        memcpy(sp->s, s, sizeof s);
        memcpy(sp->s0, s, sizeof s);
        sp->o = o;
        sp->gs = 1;
        double kappa = -2.0 * log(opt->p_min / o);
        sp->kappa = kappa;
        if (fabs(kappa) <= 1e-12) sp->hazard |= ORC_HZ_CULL;
        if (!(kappa > 0.0)) {
            sp->cull = ORC_CULL_KAPPA;
            return;
        }
        double iz = 1.0 / mu[2];
        double J[6] = {cam->fx * iz, 0.0, -cam->fx * mu[0] * iz * iz, 0.0, cam->fy * iz, -cam->fy * mu[1] * iz * iz};
        double Sig[9], RS[9], RpT[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                RS[3 * r + c] = sp->Rp[3 * r + c] * s[c] * s[c];
                RpT[3 * r + c] = sp->Rp[3 * c + r];
            }
        mat3_mul(RS, RpT, Sig);
        double JS[6];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c)
                JS[3 * r + c] = J[3 * r] * Sig[c] + J[3 * r + 1] * Sig[3 + c] + J[3 * r + 2] * Sig[6 + c];
        double P00 = JS[0] * J[0] + JS[1] * J[1] + JS[2] * J[2];
        double P01 = JS[0] * J[3] + JS[1] * J[4] + JS[2] * J[5];
        double P11 = JS[3] * J[3] + JS[4] * J[4] + JS[5] * J[5];
        double det = P00 * P11 - P01 * P01;
        if (!(det > 0.0)) {
            sp->cull = ORC_CULL_INVALID;
            return;
        }
        sp->gs_A[0] = P11 / det;
        sp->gs_A[1] = -P01 / det;
        sp->gs_A[2] = P00 / det;
        double uc = cam->fx * mu[0] * iz + cam->cx, vc = cam->fy * mu[1] * iz + cam->cy;
        sp->gs_c[0] = uc;
        sp->gs_c[1] = vc;
        /* the support ellipse (d^T Sigma_pi^-1 d <= kappa) and its box */
        double eu = sqrt(kappa * P00), ev = sqrt(kappa * P11);
        sp->all_front = 1;
        box_to_pixels(sp, cam, uc - eu, uc + eu, vc - ev, vc + ev);
        if (sp->px0 > sp->px1 || sp->py0 > sp->py1) {
            sp->cull = ORC_CULL_OFFSCREEN;
            return;
        }
        const double *A = sp->gs_A;
        sp->cq[0] = A[0]; sp->cq[1] = A[1]; sp->cq[2] = A[2];
        sp->cq[3] = -(A[0] * uc + A[1] * vc);
        sp->cq[4] = -(A[1] * uc + A[2] * vc);
        sp->cq[5] = A[0] * uc * uc + 2.0 * A[1] * uc * vc + A[2] * vc * vc - kappa;
        sp->bounded = 1;
        /* the pixel box is already the ellipse's box: the binning box is the same */
        if (!binning_box(sp, opt)) return;
        sp->listed = 0;
        for (int ty = sp->ty0; ty <= sp->ty1; ++ty)
            for (int tx = sp->tx0; tx <= sp->tx1; ++tx) sp->listed += tile_listed(sp, opt, tx, ty);
        if (sp->listed == 0) {
            sp->cull = ORC_CULL_NOTILE;
            return;
        }
        goto colour;
    }

    if (opt->mip == 1 || opt->mip == 3) {
        /* Sec. 5, eq. (17): Sigma^ = Sigma + sigma^2 tau^2 I with a
         * pixel-invariant tau = |mu| (unit rays) and sigma^2 the pixel area at
         * unit distance; opacity modulated by sqrt(|Sigma| c^2 / (|Sigma^| c^^2)). */
        double tb = sqrt(dot3(mu, mu));
        double sig2 = opt->mip_sigma2_px / (cam->fx * cam->fy);
        double ml[3];
        mat3t_vec(sp->Rp, mu, ml);
        double det = 1.0, deth = 1.0, c2p = 0.0, c2h = 0.0, sh2[3];
        for (int k = 0; k < 3; ++k) {
            double s2 = s[k] * s[k];
            sh2[k] = s2 + sig2 * tb * tb;
            det *= s2;
            deth *= sh2[k];
            c2p += ml[k] * ml[k] / s2;
            c2h += ml[k] * ml[k] / sh2[k];
        }
        /* mip = 3: the widening alone (the dilation-only ablation of Sec. 6.2) */
        if (opt->mip == 1) o = o * sqrt(det * c2p / (deth * c2h));
        for (int k = 0; k < 3; ++k) s[k] = sqrt(sh2[k]);
    }
    memcpy(sp->s, s, sizeof s);
    memcpy(sp->s0, s, sizeof s);
    sp->o = o;

    /* kappa = -2 log(p_min / o), eq. (3); skip when kappa <= 0 */
    double kappa = -2.0 * log(opt->p_min / o);
    sp->kappa = kappa;
    if (fabs(kappa) <= 1e-12) sp->hazard |= ORC_HZ_CULL;
    if (!(kappa > 0.0)) {
        sp->cull = ORC_CULL_KAPPA;
        return;
    }

    if (opt->mip == 2) {
        /* exact MIP: the quad, box and tiles below are those of the bounding
         * Gaussian; the weight is evaluated per ray with the scales s0 */
        sp->exact = 1;
        sp->sig2 = opt->mip_sigma2_px / (cam->fx * cam->fy);
        /* the camera-inside skip (eq. 6) applies to the Gaussian itself, as
         * without MIP; a bound that holds the camera gives no quad, and
         * then, as when there is no bound, the whole view is listed */
        double ml0[3], c2g = 0.0, c2b = 0.0;
        mat3t_vec(sp->Rp, mu, ml0);
        for (int k = 0; k < 3; ++k) c2g += ml0[k] * ml0[k] / (s[k] * s[k]);
        if (fabs(c2g - kappa) <= 1e-12 * c2g) sp->hazard |= ORC_HZ_CULL;
        if (!(c2g > kappa)) {
            sp->c2 = c2g;
            sp->cull = ORC_CULL_INSIDE;
            return;
        }
        double amax = mip_exact_bound(mu, s, kappa, sp->sig2);
        if (amax >= 0.0)
            for (int k = 0; k < 3; ++k) c2b += ml0[k] * ml0[k] / (s[k] * s[k] + amax);
        if (amax < 0.0 || !(c2b > kappa)) {
            sp->whole = 1;
        } else {
            for (int k = 0; k < 3; ++k) s[k] = sqrt(s[k] * s[k] + amax);
            memcpy(sp->s, s, sizeof s);
        }
    }

    /* c^2 = mu^T Sigma^-1 mu, eq. (6); skip when c^2 <= kappa (Prop. A.2) */
    double ml[3], mw[3];
    mat3t_vec(sp->Rp, mu, ml);
    for (int k = 0; k < 3; ++k) mw[k] = ml[k] / s[k];
    double c2 = dot3(mw, mw);
    sp->c2 = c2;
    memcpy(sp->mu_w, mw, sizeof mw);
    if (fabs(c2 - kappa) <= 1e-12 * c2) sp->hazard |= ORC_HZ_CULL;
    if (!(c2 > kappa)) {
        sp->cull = ORC_CULL_INSIDE;
        return;
    }
    if (sp->whole) {
        /* no bounding Gaussian: every tile of the view is listed */
        sp->all_front = 0;
        sp->bbox[0] = -INFINITY; sp->bbox[1] = INFINITY; sp->bbox[2] = -INFINITY; sp->bbox[3] = INFINITY;
        sp->px0 = 0; sp->px1 = cam->width - 1; sp->py0 = 0; sp->py1 = cam->height - 1;
        sp->bounded = 0;
        (void)binning_box(sp, opt); /* unbounded: the whole view */
        sp->listed = (sp->tx1 + 1) * (sp->ty1 + 1);
        goto colour;
    }

    /* Sec. 4.1: mu^ = S^-1 R_p^T mu / c, b = sqrt(1 - kappa/c^2),
     * Q = R_p S R_{mu^<-v}, B = Q_{0:2}^T Q_{0:2}. */
    double c = sqrt(c2);
    double muh[3] = {mw[0] / c, mw[1] / c, mw[2] / c};
    double b = sqrt(1.0 - kappa / c2);
    sp->b = b;
    orc_rot_mu_v(muh, sp->Rv);
    double RpS[9];
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) RpS[3 * r + cc] = sp->Rp[3 * r + cc] * s[cc];
    double Q[9];
    mat3_mul(RpS, sp->Rv, Q);
    double Ba = 0, Bh = 0, Bd = 0;
    for (int r = 0; r < 3; ++r) {
        Ba += Q[3 * r] * Q[3 * r];
        Bh += Q[3 * r] * Q[3 * r + 1];
        Bd += Q[3 * r + 1] * Q[3 * r + 1];
    }
    /* eq. (14): u1 = top eigenvector of the 2x2 B in closed form; u0 is u1
     * turned 90 degrees anticlockwise.  Near-isotropic B (relative eigen-gap
     * <= 1e-6) takes u1 = (1, 0). */
    double mean = 0.5 * (Ba + Bd);
    double rad = sqrt(0.25 * (Ba - Bd) * (Ba - Bd) + Bh * Bh);
    double lmax = mean + rad;
    double gap = 2.0 * rad;
    double u1[2];
    if (gap <= 1e-6 * lmax) {
        u1[0] = 1.0;
        u1[1] = 0.0;
    } else {
        double v1[2] = {Bh, lmax - Ba}, v2[2] = {lmax - Bd, Bh};
        double n1 = sqrt(v1[0] * v1[0] + v1[1] * v1[1]), n2 = sqrt(v2[0] * v2[0] + v2[1] * v2[1]);
        if (n1 >= n2) {
            u1[0] = v1[0] / n1;
            u1[1] = v1[1] / n1;
        } else {
            u1[0] = v2[0] / n2;
            u1[1] = v2[1] / n2;
        }
    }
    if (gap >= 0.5e-6 * lmax && gap <= 2e-6 * lmax) sp->hazard |= ORC_HZ_EIGEN;
    double u0[2] = {-u1[1], u1[0]};
    sp->U[0] = u0[0]; sp->U[1] = u1[0];
    sp->U[2] = u0[1]; sp->U[3] = u1[1];

    /* eq. (15): V_ray = [Q_{0:2} U_ray, mu] H(Z_ray), Z_ray = (sqrt(kappa)/b) O,
     * O = [[-1,-1,1,1],[-1,1,1,-1]] (the canonical quad of Sec. 3.3). */
    const double O[2][4] = {{-1, -1, 1, 1}, {-1, 1, 1, -1}};
    double hs = sqrt(kappa) / b;
    double QU[6]; /* 3x2 */
    for (int r = 0; r < 3; ++r) {
        QU[2 * r] = Q[3 * r] * u0[0] + Q[3 * r + 1] * u0[1];
        QU[2 * r + 1] = Q[3 * r] * u1[0] + Q[3 * r + 1] * u1[1];
    }
    int all_front = 1;
    double zmin = INFINITY, zscale = 0.0;
    for (int k = 0; k < 4; ++k) {
        double z0 = hs * O[0][k], z1 = hs * O[1][k];
        for (int r = 0; r < 3; ++r) sp->quad[3 * k + r] = QU[2 * r] * z0 + QU[2 * r + 1] * z1 + mu[r];
        double vz = sp->quad[3 * k + 2];
        if (!(vz > 0.0)) all_front = 0;
        zmin = fmin(zmin, fabs(vz));
        zscale = fmax(zscale, fabs(mu[2]) + fabs(QU[4] * z0) + fabs(QU[5] * z1));
    }
    if (zmin <= 1e-12 * zscale) sp->hazard |= ORC_HZ_FRONT;
    sp->all_front = all_front;

    /* Bounding box of the projected quad.  The quad is never clipped for
     * drawing (Sec. 4.1): every pixel of the box is still evaluated exactly.
     * When a vertex lies at z <= 0 only the box is bounded, by the part of
     * the quad inside the view frustum. */
    int W_ = cam->width, H_ = cam->height;
    int px0, px1, py0, py1;
    if (all_front) {
        double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        for (int k = 0; k < 4; ++k) {
            const double *V = &sp->quad[3 * k];
            double u = cam->fx * V[0] / V[2] + cam->cx;
            double v = cam->fy * V[1] / V[2] + cam->cy;
            umin = fmin(umin, u); umax = fmax(umax, u);
            vmin = fmin(vmin, v); vmax = fmax(vmax, v);
        }
        box_to_pixels(sp, cam, umin, umax, vmin, vmax);
        px0 = sp->px0; px1 = sp->px1; py0 = sp->py0; py1 = sp->py1;
    } else {
        /* only the box is bounded, by the part of the quad inside the view
         * frustum; the quad is never clipped for drawing */
        double cb[4];
        int cr = clip_quad_to_view(sp->quad, cam, cb);
        if (cr > 0) {
            box_to_pixels(sp, cam, cb[0], cb[1], cb[2], cb[3]);
            px0 = sp->px0; px1 = sp->px1; py0 = sp->py0; py1 = sp->py1;
        } else if (cr == 0) {
            px0 = 1; px1 = 0; py0 = 1; py1 = 0;
        } else {
            sp->bbox[0] = -INFINITY; sp->bbox[1] = INFINITY; sp->bbox[2] = -INFINITY; sp->bbox[3] = INFINITY;
            px0 = 0; px1 = W_ - 1; py0 = 0; py1 = H_ - 1;
        }
    }
    sp->px0 = px0; sp->px1 = px1; sp->py0 = py0; sp->py1 = py1;
    if (px0 > px1 || py0 > py1) {
        sp->cull = ORC_CULL_OFFSCREEN;
        return;
    }
    support_conic(sp, cam);
    if (!binning_box(sp, opt)) return;
    sp->listed = 0;
    for (int ty = sp->ty0; ty <= sp->ty1; ++ty)
        for (int tx = sp->tx0; tx <= sp->tx1; ++tx) sp->listed += tile_listed(sp, opt, tx, ty);
    if (sp->listed == 0) {
        sp->cull = ORC_CULL_NOTILE;
        return;
    }

colour:;
    /* colour: SH at the unit direction from the camera centre to the mean */
    double Cw[3]; /* camera centre = -W^T t */
    mat3t_vec(Wr, t, Cw);
    double dv[3] = {m[0] + Cw[0], m[1] + Cw[1], m[2] + Cw[2]};
    double dn = sqrt(dot3(dv, dv));
    sp->dist = dn;
    for (int k = 0; k < 3; ++k) sp->dir[k] = dv[k] / dn;
    double Y[16];
    orc_sh_basis(sc->sh_degree, sp->dir, Y, NULL);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < nk; ++k) acc += Y[k] * sc->sh[((int64_t)k * 3 + ch) * n + i];
        sp->rgb_raw[ch] = acc + 0.5;
        sp->rgb[ch] = sp->rgb_raw[ch] > 0.0 ? sp->rgb_raw[ch] : 0.0;
    }
    sp->cull = ORC_VISIBLE;
}

typedef struct {
    const orc_scene *sc;
    const orc_camera *cam;
    const orc_options *opt;
    orc_splat *out;
    int64_t begin, end;
} prep_job;

static void *prep_worker(void *arg)
{
    prep_job *j = (prep_job *)arg;
    for (int64_t i = j->begin; i < j->end; ++i) preprocess_one(j->sc, i, j->cam, j->opt, &j->out[i]);
    return NULL;
}

static int clamp_threads(int nthreads)
{
    if (nthreads < 1) return 1;
    return nthreads > 256 ? 256 : nthreads;
}

int orc_preprocess(const orc_scene *sc, const orc_camera *cam, const orc_options *opt, orc_splat *out, int nthreads)
{
    nthreads = clamp_threads(nthreads);
    pthread_t th[256];
    prep_job jobs[256];
    int64_t chunk = (sc->n + nthreads - 1) / nthreads;
    int used = 0;
    for (int k = 0; k < nthreads; ++k) {
        jobs[k] = (prep_job){sc, cam, opt, out, k * chunk, (k + 1) * chunk < sc->n ? (k + 1) * chunk : sc->n};
        if (jobs[k].begin >= jobs[k].end) break;
        pthread_create(&th[k], NULL, prep_worker, &jobs[k]);
        ++used;
    }
    for (int k = 0; k < used; ++k) pthread_join(th[k], NULL);
    return 0;
}

/* ------------------------------------------------------------- ordering */
typedef struct {
    uint32_t key;
    int64_t idx;
} key_idx;

static int cmp_key_idx(const void *a, const void *b)
{
    const key_idx *x = (const key_idx *)a, *y = (const key_idx *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Visible Gaussians in ascending (depth key, index) order (Sec. 3, eq. 1). */
static int64_t depth_order(const orc_splat *sp, int64_t n, int64_t *order)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) m += sp[i].cull == ORC_VISIBLE;
    key_idx *ki = (key_idx *)malloc(sizeof(key_idx) * (m ? m : 1));
    m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (sp[i].cull == ORC_VISIBLE) ki[m++] = (key_idx){sp[i].depth_key, i};
    qsort(ki, (size_t)m, sizeof(key_idx), cmp_key_idx);
    for (int64_t k = 0; k < m; ++k) order[k] = ki[k].idx;
    free(ki);
    return m;
}

/* Per-row candidate lists: for each row, the ordered Gaussians whose pixel box
 * spans it.  A filter that keeps the depth order; no other reordering. */
typedef struct {
    int64_t *start; /* [H + 1] */
    int64_t *items;
} row_lists;

static void build_rows(const orc_splat *sp, const int64_t *order, int64_t m, int H, row_lists *rl)
{
    rl->start = (int64_t *)calloc((size_t)H + 1, sizeof(int64_t));
    for (int64_t k = 0; k < m; ++k) {
        const orc_splat *s = &sp[order[k]];
        for (int y = s->py0; y <= s->py1; ++y) rl->start[y + 1]++;
    }
    for (int y = 0; y < H; ++y) rl->start[y + 1] += rl->start[y];
    rl->items = (int64_t *)malloc(sizeof(int64_t) * (rl->start[H] ? rl->start[H] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)H + 1));
    memcpy(fill, rl->start, sizeof(int64_t) * ((size_t)H + 1));
    for (int64_t k = 0; k < m; ++k) {
        const orc_splat *s = &sp[order[k]];
        for (int y = s->py0; y <= s->py1; ++y) rl->items[fill[y]++] = order[k];
    }
    free(fill);
}

static void free_rows(row_lists *rl)
{
    free(rl->start);
    free(rl->items);
}

/* Does the ray x hit the 3D quad of splat s in front of the camera?  (The
 * fragments a rasteriser would shade for this quad.) */
static int ray_hits_quad(const orc_splat *s, const double *x)
{
    double xl[3], xw[3];
    if (s->whole || s->gs) return 1; /* no quad: every pixel of the box */
    mat3t_vec(s->Rp, x, xl);
    for (int k = 0; k < 3; ++k) xw[k] = xl[k] / s->s[k];
    double den = dot3(xw, s->mu_w);
    if (!(den > 0.0)) return 0;
    double tt = s->c2 / den;
    double r[3] = {tt * xw[0] - s->mu_w[0], tt * xw[1] - s->mu_w[1], tt * xw[2] - s->mu_w[2]};
    /* plane coordinates in the R_v frame, then in the quad axes U */
    double p0 = s->Rv[0] * r[0] + s->Rv[3] * r[1] + s->Rv[6] * r[2];
    double p1 = s->Rv[1] * r[0] + s->Rv[4] * r[1] + s->Rv[7] * r[2];
    double z0 = s->U[0] * p0 + s->U[2] * p1;
    double z1 = s->U[1] * p0 + s->U[3] * p1;
    double hs = sqrt(s->kappa) / s->b;
    return fabs(z0) <= hs && fabs(z1) <= hs;
}

/* Margins inside which a per-pixel decision is taken within rounding distance
 * of the renderer's FP32 arithmetic (a hazard); both outcomes are then
 * correct results (several results are correct there):
 *   omega >= p_min: |ln omega - ln p_min| < 1e-4.  The FP32 divergence carries
 *     a relative error of order 1e-6 of D (about 11 at the threshold), i.e.
 *     about 6e-6 in ln omega; the margin leaves a factor of about 15;
 *   termination T' < t_eps: |ln T' - ln t_eps| < 1e-3.  ln T' sums ln(1 - a)
 *     over every contribution, each off by a / (1 - a) times the relative
 *     error of omega (up to 100 times it below the clamp);
 *   tau > 0 (Prop. A.3): the cosine between the whitened ray and the whitened
 *     centre within 1e-5 of zero. */
#define ORC_MARGIN_OMEGA 1e-4
#define ORC_MARGIN_T 1e-3
#define ORC_MARGIN_TAU 1e-5

/* cosine between S^-1 R_p^T x and S^-1 R_p^T mu (its sign is that of tau) */
static double front_cosine(const double *mu, const double *Rp, const double *s, const double *x)
{
    double xl[3], ml[3], xw[3], mw[3];
    mat3t_vec(Rp, x, xl);
    mat3t_vec(Rp, mu, ml);
    for (int k = 0; k < 3; ++k) {
        xw[k] = xl[k] / s[k];
        mw[k] = ml[k] / s[k];
    }
    return dot3(xw, mw) / sqrt(dot3(xw, xw) * dot3(mw, mw));
}

/* Rendered opacity of splat s on the ray x through pixel (px, py): omega of
 * eq. (2) with D_ray (eq. 5), D_gs (Sec. 3.1) or the exact MIP weight.
 * *front: the peak of the density along the ray lies in front of the camera
 * (tau > 0; always for D_gs); *front_hz: that sign is within ORC_MARGIN_TAU. */
static double pixel_weight(const orc_splat *s, int px, int py, const double *x, int *front, int *front_hz)
{
    double tau;
    if (s->gs) {
        double du = px + 0.5 - s->gs_c[0], dv = py + 0.5 - s->gs_c[1];
        double D = s->gs_A[0] * du * du + 2.0 * s->gs_A[1] * du * dv + s->gs_A[2] * dv * dv;
        *front = 1;
        *front_hz = 0;
        return s->o * exp(-0.5 * D);
    }
    double w, cosv;
    if (s->exact) {
        w = orc_mip_exact_weight(s->mu, s->Rp, s->s0, s->o, s->sig2, x, &tau);
        /* the peak of the widened density: its scales are those of the ray */
        double nx = sqrt(dot3(x, x)), t0, sh[3];
        orc_divergence(s->mu, s->Rp, s->s0, x, &t0, NULL);
        double a = s->sig2 / (nx * nx * nx) * (t0 * nx) * (t0 * nx);
        for (int k = 0; k < 3; ++k) sh[k] = sqrt(s->s0[k] * s->s0[k] + a);
        cosv = front_cosine(s->mu, s->Rp, sh, x);
    } else {
        double D = orc_divergence(s->mu, s->Rp, s->s, x, &tau, NULL);
        w = s->o * exp(-0.5 * D);
        cosv = front_cosine(s->mu, s->Rp, s->s, x);
    }
    *front = tau > 0.0;
    *front_hz = fabs(cosv) < ORC_MARGIN_TAU;
    return w;
}

/* Outcomes of one list entry at a pixel (eqs. 1-2 with the readings of the
 * file header): skipped (no contribution), taken, or the stop before it. */
enum { OUT_SKIP = 1, OUT_TAKE = 2, OUT_STOP = 4 };

/* The set of outcomes of entry s at transmittance T that are correct within
 * the margins (bits OUT_*); *natural receives the outcome of the decisions
 * as computed and *alpha the clamped opacity. */
static int entry_outcomes(const orc_splat *s, int px, int py, const double *x, const orc_options *opt, double T,
                          int *natural, double *alpha)
{
    int front, front_hz;
    double w = pixel_weight(s, px, py, x, &front, &front_hz);
    int pass = w >= opt->p_min;
    int pass_hz = fabs(log(w / opt->p_min)) < ORC_MARGIN_OMEGA;
    int can_contrib = (front || front_hz) && (pass || pass_hz);
    int can_skip = !front || front_hz || !pass || pass_hz;
    double a = w < opt->alpha_max ? w : opt->alpha_max;
    int set = can_skip ? OUT_SKIP : 0;
    *natural = OUT_SKIP;
    *alpha = a;
    if (can_contrib) {
        double Tn = T * (1.0 - a);
        int stop = Tn < opt->t_eps;
        int stop_hz = fabs(log(Tn / opt->t_eps)) < ORC_MARGIN_T;
        set |= stop ? OUT_STOP : OUT_TAKE;
        if (stop_hz) set |= stop ? OUT_TAKE : OUT_STOP;
        if (front && pass) *natural = stop ? OUT_STOP : OUT_TAKE;
    }
    return set;
}

typedef struct {
    double rgb[3], T;
    int32_t n_contrib;
    int32_t hazard;
    int64_t fragments, in_box, contributions;
} pixel_result;

typedef struct {
    int64_t k;      /* list position whose outcome is forced */
    double T, C[3];
    int32_t entry, last;
    int32_t outcome;
} walk_state;

#define ORC_WALK_STACK 64

/* Composite one pixel (eqs. 1-2) over the candidate list cand[0..nc) in
 * depth order; an entry counts when the pixel lies in its box.  *res gets the
 * result of the decisions as computed, with res->hazard = 1 when any of them
 * on its path lies within its margin.  With leaves != NULL every combination
 * of the outcomes of such decisions is followed as well, and the pixel values
 * (r, g, b, T) of every path are written to leaves[0..) (leaves[0] is the
 * computed one), at most cap of them; returns their number, or -1 when there
 * are more. */
static int walk_pixel(const orc_splat *sp, const int64_t *cand, int64_t nc, int px, int py, const orc_camera *cam,
                      const orc_options *opt, pixel_result *res, double *leaves, int cap)
{
    const double x[3] = {(px + 0.5 - cam->cx) / cam->fx, (py + 0.5 - cam->cy) / cam->fy, 1.0};
    walk_state stack[ORC_WALK_STACK];
    int top = 0, n_leaves = 0, overflow = 0, primary = 1;
    walk_state st = {0, 1.0, {0.0, 0.0, 0.0}, 0, 0, 0};
    int64_t frags = 0, inbox = 0, contrib = 0;
    int32_t hz = 0;
    for (;;) {
        int64_t k = st.k;
        double T = st.T, C[3] = {st.C[0], st.C[1], st.C[2]};
        int32_t entry = st.entry, last = st.last;
        int forced = st.outcome;
        for (; k < nc; ++k) {
            const orc_splat *s = &sp[cand[k]];
            if (px < s->px0 || px > s->px1 || py < s->py0 || py > s->py1) continue;
            int natural, outcome;
            double a;
            int set = entry_outcomes(s, px, py, x, opt, T, &natural, &a);
            if (forced) {
                outcome = forced; /* entry k was counted when this state was saved */
                forced = 0;
            } else {
                ++entry;
                if (primary) {
                    ++inbox;
                    frags += ray_hits_quad(s, x);
                }
                if (set != natural) {
                    if (primary) hz = 1;
                    for (int o = OUT_SKIP; leaves && o <= OUT_STOP; o <<= 1) {
                        if (!(set & o) || o == natural) continue;
                        if (top == ORC_WALK_STACK) {
                            overflow = 1;
                            continue;
                        }
                        stack[top++] = (walk_state){k, T, {C[0], C[1], C[2]}, entry, last, o};
                    }
                }
                outcome = natural;
            }
            if (outcome == OUT_STOP) break;
            if (outcome == OUT_TAKE) {
                for (int ch = 0; ch < 3; ++ch) C[ch] += T * a * s->rgb[ch];
                T = T * (1.0 - a);
                last = entry;
                if (primary) ++contrib;
            }
        }
        double out[4];
        for (int ch = 0; ch < 3; ++ch) out[ch] = C[ch] + T * opt->background[ch];
        out[3] = T;
        if (primary) {
            for (int ch = 0; ch < 3; ++ch) res->rgb[ch] = out[ch];
            res->T = T;
            res->n_contrib = last;
            res->hazard = hz;
            res->fragments = frags;
            res->in_box = inbox;
            res->contributions = contrib;
            primary = 0;
        }
        if (!leaves) break;
        if (n_leaves < cap)
            memcpy(leaves + 4 * n_leaves++, out, sizeof out);
        else
            overflow = 1;
        if (top == 0) break;
        st = stack[--top];
    }
    return leaves ? (overflow ? -1 : n_leaves) : 1;
}

typedef struct {
    const orc_splat *sp;
    const row_lists *rl;
    const orc_camera *cam;
    const orc_options *opt;
    int y_begin, y_end, stride, offset;
    double *rgb, *T;
    uint8_t *hazard;
    int32_t *n_contrib;
    int64_t frags, inbox, contrib;
} render_job;

static void *render_worker(void *arg)
{
    render_job *j = (render_job *)arg;
    const int W = j->cam->width, H = j->cam->height;
    for (int y = j->y_begin + j->offset; y < j->y_end; y += j->stride) {
        const int64_t *cand = j->rl->items + j->rl->start[y];
        int64_t nc = j->rl->start[y + 1] - j->rl->start[y];
        for (int x = 0; x < W; ++x) {
            pixel_result r;
            walk_pixel(j->sp, cand, nc, x, y, j->cam, j->opt, &r, NULL, 0);
            int64_t p = (int64_t)y * W + x;
            for (int ch = 0; ch < 3; ++ch) j->rgb[(int64_t)ch * H * W + p] = r.rgb[ch];
            j->T[p] = r.T;
            if (j->hazard) j->hazard[p] = (uint8_t)r.hazard;
            if (j->n_contrib) j->n_contrib[p] = r.n_contrib;
            j->frags += r.fragments;
            j->inbox += r.in_box;
            j->contrib += r.contributions;
        }
    }
    return NULL;
}

/* Render rows [y_begin, y_end) of one view.  rgb is [3][H][W], T / hazard /
 * n_contrib are [H][W]; rows outside the range are left untouched.
 * counters (optional, 5 entries): visible Gaussians, instances (Gaussian-tile
 * pairs), fragments (pixel centre inside a projected quad), pixel-box pairs,
 * contributions -- the last three over the rendered rows only. */
int orc_render(const orc_scene *sc, const orc_camera *cam, const orc_options *opt, int y_begin, int y_end,
               int nthreads, double *rgb, double *T, uint8_t *hazard, int32_t *n_contrib, int64_t *counters)
{
    nthreads = clamp_threads(nthreads);
    int64_t n = sc->n;
    orc_splat *sp = (orc_splat *)malloc(sizeof(orc_splat) * (n ? n : 1));
    orc_preprocess(sc, cam, opt, sp, nthreads);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t m = depth_order(sp, n, order);
    row_lists rl;
    build_rows(sp, order, m, cam->height, &rl);
    if (y_begin < 0) y_begin = 0;
    if (y_end > cam->height) y_end = cam->height;
    pthread_t th[256];
    render_job jobs[256];
    for (int k = 0; k < nthreads; ++k) {
        jobs[k] = (render_job){sp, &rl, cam, opt, y_begin, y_end, nthreads, k, rgb, T, hazard, n_contrib, 0, 0, 0};
        pthread_create(&th[k], NULL, render_worker, &jobs[k]);
    }
    int64_t frags = 0, inbox = 0, contrib = 0;
    for (int k = 0; k < nthreads; ++k) {
        pthread_join(th[k], NULL);
        frags += jobs[k].frags;
        inbox += jobs[k].inbox;
        contrib += jobs[k].contrib;
    }
    if (counters) {
        int64_t inst = 0;
        for (int64_t k = 0; k < m; ++k) inst += sp[order[k]].listed;
        counters[0] = m;
        counters[1] = inst;
        counters[2] = frags;
        counters[3] = inbox;
        counters[4] = contrib;
    }
    free_rows(&rl);
    free(order);
    free(sp);
    return 0;
}

typedef struct {
    const orc_splat *sp;
    const row_lists *rl;
    const orc_camera *cam;
    const orc_options *opt;
    const int32_t *px, *py;
    int64_t begin, end;
    double *rgb, *T;
    uint8_t *hazard;
    double *leaves;
    int32_t *n_leaves;
    int cap;
} pixels_job;

static void *pixels_worker(void *arg)
{
    pixels_job *j = (pixels_job *)arg;
    for (int64_t k = j->begin; k < j->end; ++k) {
        int x = j->px[k], y = j->py[k];
        pixel_result r;
        double *lv = j->leaves ? j->leaves + 4 * (int64_t)j->cap * k : NULL;
        int nl = 0;
        if (x >= 0 && x < j->cam->width && y >= 0 && y < j->cam->height) {
            const int64_t *cand = j->rl->items + j->rl->start[y];
            nl = walk_pixel(j->sp, cand, j->rl->start[y + 1] - j->rl->start[y], x, y, j->cam, j->opt, &r, lv, j->cap);
        } else {
            memset(&r, 0, sizeof r);
            r.T = 1.0;
            for (int ch = 0; ch < 3; ++ch) r.rgb[ch] = j->opt->background[ch];
        }
        for (int ch = 0; ch < 3; ++ch) j->rgb[3 * k + ch] = r.rgb[ch];
        j->T[k] = r.T;
        if (j->hazard) j->hazard[k] = (uint8_t)r.hazard;
        if (j->n_leaves) j->n_leaves[k] = nl;
    }
    return NULL;
}

/* Render an arbitrary list of pixels (px[k], py[k]); rgb is [npix][3], T and
 * hazard [npix].  With leaves != NULL (npix x cap x 4 doubles) and n_leaves
 * (npix int32), every correct result of each pixel (all combinations of the
 * outcomes of decisions within their margins, see walk_pixel) is written too:
 * leaves[k][0..n_leaves[k]) as (r, g, b, T), the computed result first;
 * n_leaves[k] = -1 when a pixel has more than cap. */
int orc_render_pixels(const orc_scene *sc, const orc_camera *cam, const orc_options *opt, const int32_t *px,
                      const int32_t *py, int64_t npix, int nthreads, double *rgb, double *T, uint8_t *hazard,
                      double *leaves, int32_t *n_leaves, int cap)
{
    nthreads = clamp_threads(nthreads);
    int64_t n = sc->n;
    orc_splat *sp = (orc_splat *)malloc(sizeof(orc_splat) * (n ? n : 1));
    orc_preprocess(sc, cam, opt, sp, nthreads);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t m = depth_order(sp, n, order);
    row_lists rl;
    build_rows(sp, order, m, cam->height, &rl);
    pthread_t th[256];
    pixels_job jobs[256];
    int64_t chunk = (npix + nthreads - 1) / nthreads;
    int used = 0;
    for (int k = 0; k < nthreads; ++k) {
        int64_t b = k * chunk, e = (k + 1) * chunk < npix ? (k + 1) * chunk : npix;
        if (b >= e) break;
        jobs[k] = (pixels_job){sp, &rl, cam, opt, px, py, b, e, rgb, T, hazard, leaves, n_leaves, cap};
        pthread_create(&th[k], NULL, pixels_worker, &jobs[k]);
        ++used;
    }
    for (int k = 0; k < used; ++k) pthread_join(th[k], NULL);
    free_rows(&rl);
    free(order);
    free(sp);
    return 0;
}

/* Cells of tile (tx, ty) holding a pixel centre of the support of splat s:
 * inside its pixel box, with omega >= p_min and the peak in front of the
 * camera, both decisions clear of their margins.  The tile is cut into cells
 * of cw x ch pixels; bit cy * (tile_w / cw) + cx stands for cell (cx, cy). */
static uint32_t tile_support_cells(const orc_splat *s, const orc_camera *cam, const orc_options *opt, int tx, int ty,
                                   int cw, int ch)
{
    uint32_t cells = 0;
    const int ncx = opt->tile_w / cw;
    for (int r = 0; r < opt->tile_h; ++r) {
        int py = ty * opt->tile_h + r;
        if (py < s->py0 || py > s->py1) continue;
        for (int c = 0; c < opt->tile_w; ++c) {
            int px = tx * opt->tile_w + c;
            uint32_t bit = 1u << ((r / ch) * ncx + c / cw);
            if (px < s->px0 || px > s->px1 || (cells & bit)) continue;
            double x[3] = {(px + 0.5 - cam->cx) / cam->fx, (py + 0.5 - cam->cy) / cam->fy, 1.0};
            int front, front_hz;
            double w = pixel_weight(s, px, py, x, &front, &front_hz);
            if (front && !front_hz && w >= opt->p_min * (1.0 + ORC_MARGIN_OMEGA)) cells |= bit;
        }
    }
    return cells;
}

typedef struct {
    const orc_splat *sp;
    const orc_camera *cam;
    const orc_options *opt;
    const int64_t *tiles, *ids;
    int32_t tiles_x, cw, ch;
    int64_t begin, end;
    uint32_t *cells;
} cells_job;

static void *cells_worker(void *arg)
{
    cells_job *j = (cells_job *)arg;
    for (int64_t k = j->begin; k < j->end; ++k) {
        int tx = (int)(j->tiles[k] % j->tiles_x), ty = (int)(j->tiles[k] / j->tiles_x);
        j->cells[k] = tile_support_cells(&j->sp[j->ids[k]], j->cam, j->opt, tx, ty, j->cw, j->ch);
    }
    return NULL;
}

/* For each (tile, splat) pair k (tile = ty * tiles_x + tx of one view), the
 * cells of cw x ch pixels of the tile that hold a pixel centre of the splat's
 * support (tile_support_cells) in cells[k]; at most 32 cells per tile.  sp is
 * the output of orc_preprocess. */
int orc_support_cells(const orc_splat *sp, const orc_camera *cam, const orc_options *opt, int32_t tiles_x,
                      const int64_t *tiles, const int64_t *ids, int64_t m, int32_t cw, int32_t ch, uint32_t *cells,
                      int nthreads)
{
    if (cw < 1 || ch < 1 || opt->tile_w % cw || opt->tile_h % ch || (opt->tile_w / cw) * (opt->tile_h / ch) > 32)
        return -1;
    nthreads = clamp_threads(nthreads);
    pthread_t th[256];
    cells_job jobs[256];
    int64_t chunk = (m + nthreads - 1) / nthreads;
    int used = 0;
    for (int k = 0; k < nthreads; ++k) {
        int64_t b = k * chunk, e = (k + 1) * chunk < m ? (k + 1) * chunk : m;
        if (b >= e) break;
        jobs[k] = (cells_job){sp, cam, opt, tiles, ids, tiles_x, cw, ch, b, e, cells};
        pthread_create(&th[k], NULL, cells_worker, &jobs[k]);
        ++used;
    }
    for (int k = 0; k < used; ++k) pthread_join(th[k], NULL);
    return 0;
}

/* ------------------------------------------------------------- backward
 * Gradients of L with respect to every parameter, given dL/dC for each output
 * pixel (dL_dC is [3][H][W]; pixels whose three entries are zero are skipped).
 * Results are ADDED into the gradient arrays (same shapes as the inputs).
 * With MIP (Sec. 5, eq. 17) the rendered scales and opacity are functions of
 * the parameters and of mu (through tau = |mu|); their gradients are chained
 * through that transform per Gaussian (see mip_chain below).
 *
 * Compositing adjoint of eq. (1): with T_i the transmittance in front of
 * Gaussian i, dL/d rgb_i = T_i a_i g and
 *   dL/d a_i = T_i (rgb_i . g) - (sum_{j>i} T_j a_j (rgb_j . g) + T_final (bg . g)) / (1 - a_i).
 * a = min(omega, alpha_max): the clamp passes no gradient.  omega = o exp(-D/2).
 * D is the minimum over the ray of the Mahalanobis distance (Prop. A.1), so by
 * the envelope theorem, with e = tau x - mu:
 *   dD/dmu = -2 Sigma^-1 e,   dD/dSigma^-1 = e e^T.
 * Sigma^-1 = R_p diag(s^-2) R_p^T, R_p = W R(q/|q|), s = exp(l), mu = W m + t. */
typedef struct {
    double d_mu[3], d_Rp[9], d_l[3], d_o, d_rgb[3];
    double d_c[2], d_A[4]; /* D_gs: dL/d pi(mu) and dL/d Sigma_pi^-1 (2x2, row-major) */
} splat_grad;

/* Gradient of ln omega of the exact MIP weight (orc_mip_exact_weight) for the
 * ray xbar, times g, added into d_mu, d_Rp and d_l (log-scales).  In the
 * Gaussian's axes, with xl = R_p^T xbar, ml = R_p^T mu, the plain sums
 * P = sum xl^2/s^2 = xbar.Sigma^-1 xbar and Lp = sum ml xl/s^2, the widening
 * a = sigma^2 Lp^2 / (|xbar| P^2) (sigma_x^2 tau^2 of the unit ray), the
 * widened variances v = s^2 + a and Q = sum xl^2/v, L = sum ml xl/v,
 * tau^ = L/Q:
 *   ln omega = ln o + (1/2)(sum ln s^2 - sum ln v + ln P - ln Q) - D/2,
 *   dD/dml_k = 2 (ml_k - tau^ xl_k)/v_k, dD/dv_k = -(ml_k - tau^ xl_k)^2/v_k^2,
 *   dD/dxl_k = -2 tau^ (ml_k - tau^ xl_k)/v_k,
 * and a reaches every v_k.  Returns d ln omega / d ln o (= 1) times g. */
static double mip_exact_grad(const double *mu, const double *Rp, const double *s, double sig2, const double *xbar,
                             double g, double *d_mu, double *d_Rp, double *d_l)
{
    double xl[3], ml[3], s2[3], v[3];
    mat3t_vec(Rp, xbar, xl);
    mat3t_vec(Rp, mu, ml);
    double nx = sqrt(dot3(xbar, xbar));
    double P = 0.0, Lp = 0.0;
    for (int k = 0; k < 3; ++k) {
        s2[k] = s[k] * s[k];
        P += xl[k] * xl[k] / s2[k];
        Lp += ml[k] * xl[k] / s2[k];
    }
    double tb = Lp / P;
    double a = sig2 / nx * tb * tb;
    double Q = 0.0, L = 0.0;
    for (int k = 0; k < 3; ++k) {
        v[k] = s2[k] + a;
        Q += xl[k] * xl[k] / v[k];
        L += ml[k] * xl[k] / v[k];
    }
    double th = L / Q;
    double gv[3], gml[3], gxl[3], gs[3], ga = 0.0;
    for (int k = 0; k < 3; ++k) {
        double r = ml[k] - th * xl[k];
        gv[k] = -0.5 / v[k] + xl[k] * xl[k] / (2.0 * Q * v[k] * v[k]) + r * r / (2.0 * v[k] * v[k]);
        gml[k] = -r / v[k];
        gxl[k] = -xl[k] / (Q * v[k]) + th * r / v[k] + xl[k] / (P * s2[k]);
        gs[k] = 1.0 / s[k] - xl[k] * xl[k] / (P * s2[k] * s[k]) + gv[k] * 2.0 * s[k];
        ga += gv[k];
    }
    /* a = sig2 / nx * (Lp / P)^2 */
    double da_dLp = 2.0 * sig2 / nx * tb / P, da_dP = -2.0 * sig2 / nx * tb * tb / P;
    for (int k = 0; k < 3; ++k) {
        gml[k] += ga * da_dLp * xl[k] / s2[k];
        gxl[k] += ga * (da_dLp * ml[k] / s2[k] + da_dP * 2.0 * xl[k] / s2[k]);
        gs[k] += ga * (da_dLp * (-2.0 * ml[k] * xl[k] / (s2[k] * s[k])) + da_dP * (-2.0 * xl[k] * xl[k] / (s2[k] * s[k])));
    }
    double dmu[3];
    mat3_vec(Rp, gml, dmu);
    for (int r = 0; r < 3; ++r) {
        d_mu[r] += g * dmu[r];
        for (int k = 0; k < 3; ++k) d_Rp[3 * r + k] += g * (mu[r] * gml[k] + xbar[r] * gxl[k]);
    }
    for (int k = 0; k < 3; ++k) d_l[k] += g * gs[k] * s[k];
    return g;
}

/* D_gs (Sec. 3.1) of splat s at pixel (px, py); d receives p - pi(mu). */
static double gs_divergence(const orc_splat *s, int px, int py, double *d)
{
    d[0] = px + 0.5 - s->gs_c[0];
    d[1] = py + 0.5 - s->gs_c[1];
    return s->gs_A[0] * d[0] * d[0] + 2.0 * s->gs_A[1] * d[0] * d[1] + s->gs_A[2] * d[1] * d[1];
}

/* Chain of the linearised divergence: from dL/d pi(mu) (d_c) and
 * dL/d Sigma_pi^-1 (d_A) to dL/d mu, dL/d R_p and dL/d log s (added).
 * Sigma_pi = J Sigma J^T with J(mu) the pinhole Jacobian and
 * Sigma = R_p S^2 R_p^T: dL/dSigma_pi = -A d_A A (A = Sigma_pi^-1),
 * dL/dSigma = J^T (dL/dSigma_pi) J, dL/dJ = 2 (dL/dSigma_pi) J Sigma, and
 * pi(mu) has Jacobian J. */
static void gs_chain(const orc_splat *s, const orc_camera *cam, const double *d_c, const double *d_A, double *d_mu,
                     double *d_Rp, double *d_l)
{
    const double *mu = s->mu;
    double iz = 1.0 / mu[2];
    double J[6] = {cam->fx * iz, 0.0, -cam->fx * mu[0] * iz * iz, 0.0, cam->fy * iz, -cam->fy * mu[1] * iz * iz};
    double A[4] = {s->gs_A[0], s->gs_A[1], s->gs_A[1], s->gs_A[2]};
    double T[4], GP[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) T[2 * r + c] = d_A[2 * r] * A[c] + d_A[2 * r + 1] * A[2 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) GP[2 * r + c] = -(A[2 * r] * T[c] + A[2 * r + 1] * T[2 + c]);
    double Sig[9], RS[9], RpT[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            RS[3 * r + c] = s->Rp[3 * r + c] * s->s[c] * s->s[c];
            RpT[3 * r + c] = s->Rp[3 * c + r];
        }
    mat3_mul(RS, RpT, Sig);
    double GS[9], GJ[6];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) acc += J[3 * r + a] * GP[2 * r + c] * J[3 * c + b];
            GS[3 * a + b] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int c = 0; c < 2; ++c)
                for (int a = 0; a < 3; ++a) acc += GP[2 * r + c] * J[3 * c + a] * Sig[3 * a + b];
            GJ[3 * r + b] = 2.0 * acc;
        }
    /* pi(mu) and J(mu) */
    for (int a = 0; a < 3; ++a) d_mu[a] += J[a] * d_c[0] + J[3 + a] * d_c[1];
    d_mu[0] += GJ[2] * (-cam->fx * iz * iz);
    d_mu[1] += GJ[5] * (-cam->fy * iz * iz);
    d_mu[2] += GJ[0] * (-cam->fx * iz * iz) + GJ[2] * (2.0 * cam->fx * mu[0] * iz * iz * iz) +
               GJ[4] * (-cam->fy * iz * iz) + GJ[5] * (2.0 * cam->fy * mu[1] * iz * iz * iz);
    /* Sigma = R_p S^2 R_p^T */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j) acc += GS[3 * r + j] * s->Rp[3 * j + c];
            d_Rp[3 * r + c] += 2.0 * acc * s->s[c] * s->s[c];
        }
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) acc += s->Rp[3 * a + k] * GS[3 * a + b] * s->Rp[3 * b + k];
        d_l[k] += 2.0 * s->s[k] * s->s[k] * acc;
    }
}

/* Chain through the eq. (17) transform.  With s0 = exp(l), o0 = sigmoid(a),
 * ml = R_p^T mu, sigma^2 the pixel area at unit distance and tau^2 = |mu|^2:
 *   s_k^2 = s0_k^2 + sigma^2 tau^2,
 *   log o = log o0 + log|S0| + (1/2) log c2p - log|S| - (1/2) log c2h,
 *   c2p = sum_k ml_k^2 / s0_k^2,  c2h = sum_k ml_k^2 / s_k^2.
 * Given dL/dlog s_k (d_l) and dL/do (d_o) of the rendered values, adds the
 * gradients with respect to log s0 (d_l0), mu (d_mu) and R_p (d_Rp) and
 * returns dL/dlog o0. */
static double mip_chain(const double *mu, const double *Rp, const double *s0, const double *s, double sigma2,
                        const double *d_l, double d_o, double o, double *d_l0, double *d_mu, double *d_Rp)
{
    double ml[3];
    mat3t_vec(Rp, mu, ml);
    double c2p = 0.0, c2h = 0.0, ml2s4 = 0.0, inv_s2sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        c2p += ml[k] * ml[k] / (s0[k] * s0[k]);
        c2h += ml[k] * ml[k] / (s[k] * s[k]);
        ml2s4 += ml[k] * ml[k] / (s[k] * s[k] * s[k] * s[k]);
        inv_s2sum += 1.0 / (s[k] * s[k]);
    }
    const double Lo = d_o * o; /* dL/dlog o */
    double gmu[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        const double r = s0[k] * s0[k] / (s[k] * s[k]); /* dlog s_k / dlog s0_k */
        /* through log s_k directly and through log o (|S0|, c2p, |S|, c2h) */
        d_l0[k] += d_l[k] * r +
                   Lo * (1.0 - ml[k] * ml[k] / (s0[k] * s0[k]) / c2p - r + ml[k] * ml[k] / (s[k] * s[k]) * r / c2h);
        /* dlog s_k / dmu = sigma^2 mu / s_k^2 */
        for (int j = 0; j < 3; ++j) gmu[j] += d_l[k] * sigma2 * mu[j] / (s[k] * s[k]);
    }
    /* log o through ml (c2p, c2h) and through tau (|S| and c2h) */
    double a0[3], a1[3], v0[3], v1[3];
    for (int k = 0; k < 3; ++k) {
        a0[k] = ml[k] / (s0[k] * s0[k]);
        a1[k] = ml[k] / (s[k] * s[k]);
    }
    mat3_vec(Rp, a0, v0);
    mat3_vec(Rp, a1, v1);
    for (int j = 0; j < 3; ++j)
        gmu[j] += Lo * (v0[j] / c2p - v1[j] / c2h - sigma2 * mu[j] * inv_s2sum + sigma2 * mu[j] * ml2s4 / c2h);
    for (int j = 0; j < 3; ++j) d_mu[j] += gmu[j];
    /* ml_k = sum_r R_p[r][k] mu_r */
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) d_Rp[3 * r + k] += Lo * mu[r] * (a0[k] / c2p - a1[k] / c2h);
    return Lo;
}

int orc_backward(const orc_scene *sc, const orc_camera *cam, const orc_options *opt, const double *dL_dC,
                 double *g_means, double *g_log_scales, double *g_quats, double *g_opacity, double *g_sh)
{
    if (opt->mip == 3) return -2; /* dilation only: forward only */
    int64_t n = sc->n;
    const int W = cam->width, H = cam->height;
    orc_splat *sp = (orc_splat *)malloc(sizeof(orc_splat) * (n ? n : 1));
    orc_preprocess(sc, cam, opt, sp, 1);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t m = depth_order(sp, n, order);
    row_lists rl;
    build_rows(sp, order, m, H, &rl);
    splat_grad *gg = (splat_grad *)calloc((size_t)(n ? n : 1), sizeof(splat_grad));

    typedef struct {
        int64_t idx;
        double T, a, w, D, tau;
        int clamped;
    } contrib_rec;
    int64_t cap = 1024;
    contrib_rec *list = (contrib_rec *)malloc(sizeof(contrib_rec) * cap);

    for (int py = 0; py < H; ++py) {
        const int64_t *cand = rl.items + rl.start[py];
        int64_t nc = rl.start[py + 1] - rl.start[py];
        for (int px = 0; px < W; ++px) {
            int64_t p = (int64_t)py * W + px;
            double g[3] = {dL_dC[p], dL_dC[(int64_t)H * W + p], dL_dC[2 * (int64_t)H * W + p]};
            if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
            double x[3] = {(px + 0.5 - cam->cx) / cam->fx, (py + 0.5 - cam->cy) / cam->fy, 1.0};
            /* forward pass, recording the contributors */
            double T = 1.0;
            int64_t nl = 0;
            for (int64_t k = 0; k < nc; ++k) {
                const orc_splat *s = &sp[cand[k]];
                if (px < s->px0 || px > s->px1) continue;
                double tau = 1.0, D = 0.0, dgs[2], w;
                if (s->exact) {
                    w = orc_mip_exact_weight(s->mu, s->Rp, s->s0, s->o, s->sig2, x, &tau);
                } else {
                    if (s->gs)
                        D = gs_divergence(s, px, py, dgs);
                    else
                        D = orc_divergence(s->mu, s->Rp, s->s, x, &tau, NULL);
                    w = s->o * exp(-0.5 * D);
                }
                if (!(tau > 0.0)) continue;
                if (!(w >= opt->p_min)) continue;
                double a = w < opt->alpha_max ? w : opt->alpha_max;
                double Tn = T * (1.0 - a);
                if (Tn < opt->t_eps) break;
                if (nl == cap) {
                    cap *= 2;
                    list = (contrib_rec *)realloc(list, sizeof(contrib_rec) * cap);
                }
                list[nl++] = (contrib_rec){cand[k], T, a, w, D, tau, !(w < opt->alpha_max)};
                T = Tn;
            }
            /* reverse sweep */
            double S = T * (opt->background[0] * g[0] + opt->background[1] * g[1] + opt->background[2] * g[2]);
            for (int64_t k = nl - 1; k >= 0; --k) {
                const contrib_rec *c = &list[k];
                const orc_splat *s = &sp[c->idx];
                splat_grad *G = &gg[c->idx];
                double rg = s->rgb[0] * g[0] + s->rgb[1] * g[1] + s->rgb[2] * g[2];
                for (int ch = 0; ch < 3; ++ch) G->d_rgb[ch] += c->T * c->a * g[ch];
                double dL_da = c->T * rg - S / (1.0 - c->a);
                S += c->T * c->a * rg;
                if (c->clamped) continue;
                double dL_dw = dL_da;
                G->d_o += dL_dw * c->w / s->o;
                double dL_dD = -0.5 * c->w * dL_dw;
                if (s->exact) {
                    /* dL/d ln omega = dL/domega omega (the d_o term above is its ln o part) */
                    mip_exact_grad(s->mu, s->Rp, s->s0, s->sig2, x, dL_dw * c->w, G->d_mu, G->d_Rp, G->d_l);
                    continue;
                }
                if (s->gs) {
                    /* D_gs = d^T A d with d = p - pi(mu): dD/dpi = -2 A d, dD/dA = d d^T */
                    double d[2];
                    gs_divergence(s, px, py, d);
                    G->d_c[0] += dL_dD * (-2.0 * (s->gs_A[0] * d[0] + s->gs_A[1] * d[1]));
                    G->d_c[1] += dL_dD * (-2.0 * (s->gs_A[1] * d[0] + s->gs_A[2] * d[1]));
                    G->d_A[0] += dL_dD * d[0] * d[0];
                    G->d_A[1] += dL_dD * d[0] * d[1];
                    G->d_A[2] += dL_dD * d[1] * d[0];
                    G->d_A[3] += dL_dD * d[1] * d[1];
                    continue;
                }
                double e[3];
                orc_divergence(s->mu, s->Rp, s->s, x, NULL, e);
                double f[3], Pe[3], fs[3];
                mat3t_vec(s->Rp, e, f); /* f = R_p^T e */
                for (int k2 = 0; k2 < 3; ++k2) fs[k2] = f[k2] / (s->s[k2] * s->s[k2]);
                mat3_vec(s->Rp, fs, Pe); /* Sigma^-1 e */
                for (int k2 = 0; k2 < 3; ++k2) G->d_mu[k2] += dL_dD * (-2.0 * Pe[k2]);
                /* dD = e^T dSigma^-1 e with dSigma^-1 = dR_p L R_p^T + R_p dL R_p^T + R_p L dR_p^T */
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) G->d_Rp[3 * r + cc] += dL_dD * 2.0 * e[r] * fs[cc];
                for (int k2 = 0; k2 < 3; ++k2) G->d_l[k2] += dL_dD * (-2.0 * f[k2] * f[k2] / (s->s[k2] * s->s[k2]));
            }
        }
    }

    /* chain per Gaussian to the parameters */
    const double *Wm = cam->w2c;
    double Wr[9] = {Wm[0], Wm[1], Wm[2], Wm[4], Wm[5], Wm[6], Wm[8], Wm[9], Wm[10]};
    int nk = (sc->sh_degree + 1) * (sc->sh_degree + 1);
    for (int64_t i = 0; i < n; ++i) {
        const orc_splat *s = &sp[i];
        if (s->cull != ORC_VISIBLE) continue;
        const splat_grad *G = &gg[i];
        double d_mu[3], d_Rp[9], d_l0[3], Lo;
        const double o0 = 1.0 / (1.0 + exp(-sc->opacity_logits[i]));
        memcpy(d_mu, G->d_mu, sizeof d_mu);
        memcpy(d_Rp, G->d_Rp, sizeof d_Rp);
        if (s->gs) {
            for (int k = 0; k < 3; ++k) d_l0[k] = G->d_l[k];
            gs_chain(s, cam, G->d_c, G->d_A, d_mu, d_Rp, d_l0);
            Lo = G->d_o * s->o;
        } else if (opt->mip == 1) {
            const double s0[3] = {exp(sc->log_scales[i]), exp(sc->log_scales[n + i]), exp(sc->log_scales[2 * n + i])};
            for (int k = 0; k < 3; ++k) d_l0[k] = 0.0;
            Lo = mip_chain(s->mu, s->Rp, s0, s->s, opt->mip_sigma2_px / (cam->fx * cam->fy), G->d_l, G->d_o, s->o,
                           d_l0, d_mu, d_Rp);
        } else {
            /* log-scales (s = exp(l) enters Sigma^-1 only) */
            for (int k = 0; k < 3; ++k) d_l0[k] = G->d_l[k];
            Lo = G->d_o * s->o;
        }
        /* means through mu = W m + t */
        double dm[3];
        mat3t_vec(Wr, d_mu, dm);
        for (int k = 0; k < 3; ++k) g_log_scales[k * n + i] += d_l0[k];
        /* rotation: dL/dR = W^T dL/dR_p, then the quaternion */
        double dR[9];
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc)
                dR[3 * r + cc] = Wr[r] * d_Rp[cc] + Wr[3 + r] * d_Rp[3 + cc] + Wr[6 + r] * d_Rp[6 + cc];
        double q[4];
        for (int k = 0; k < 4; ++k) q[k] = sc->quats[k * n + i];
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
        /* partial derivatives of R(w,x,y,z) entry by entry */
        double dq[4] = {0, 0, 0, 0};
        const double J[9][4] = {
            {0, 0, -4 * y, -4 * z},          {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
            {2 * z, 2 * y, 2 * x, 2 * w},    {0, -4 * x, 0, -4 * z},         {-2 * x, -2 * w, 2 * z, 2 * y},
            {-2 * y, 2 * z, -2 * w, 2 * x},  {2 * x, 2 * w, 2 * z, 2 * y},   {0, -4 * x, -4 * y, 0}};
        for (int e = 0; e < 9; ++e)
            for (int k = 0; k < 4; ++k) dq[k] += dR[e] * J[e][k];
        double qh[4] = {w, x, y, z};
        double proj = qh[0] * dq[0] + qh[1] * dq[1] + qh[2] * dq[2] + qh[3] * dq[3];
        for (int k = 0; k < 4; ++k) g_quats[k * n + i] += (dq[k] - qh[k] * proj) / qn;
        /* opacity logit: dlog o0 / da = 1 - o0 */
        g_opacity[i] += Lo * (1.0 - o0);
        /* SH coefficients and the view direction */
        double Y[16], dY[48];
        orc_sh_basis(sc->sh_degree, s->dir, Y, dY);
        double ddir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) {
            if (!(s->rgb_raw[ch] > 0.0)) continue;
            double gc = G->d_rgb[ch];
            for (int k = 0; k < nk; ++k) {
                g_sh[((int64_t)k * 3 + ch) * n + i] += Y[k] * gc;
                double coef = sc->sh[((int64_t)k * 3 + ch) * n + i];
                for (int j = 0; j < 3; ++j) ddir[j] += gc * coef * dY[3 * k + j];
            }
        }
        double pd = dot3(ddir, s->dir);
        for (int j = 0; j < 3; ++j) dm[j] += (ddir[j] - s->dir[j] * pd) / s->dist;
        for (int k = 0; k < 3; ++k) g_means[k * n + i] += dm[k];
    }
    free(list);
    free(gg);
    free_rows(&rl);
    free(order);
    free(sp);
    return 0;
}

/* (tile, Gaussian) pairs of every listed tile of the visible splats, in
 * Gaussian index order and row-major tile order; tiles[] receives
 * ty * tiles_x + tx.  Returns the number of pairs written (at most cap). */
int64_t orc_list_tiles(orc_splat *sp, int64_t n, const orc_options *opt, int32_t tiles_x, int64_t *tiles,
                       int64_t *ids, int64_t cap)
{
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        orc_splat *s = &sp[i];
        if (s->cull != ORC_VISIBLE) continue;
        for (int ty = s->ty0; ty <= s->ty1; ++ty)
            for (int tx = s->tx0; tx <= s->tx1; ++tx)
                if (tile_listed(s, opt, tx, ty) && w < cap) {
                    tiles[w] = (int64_t)ty * tiles_x + tx;
                    ids[w] = i;
                    ++w;
                }
    }
    return w;
}

int orc_splat_size(void) { return (int)sizeof(orc_splat); }
