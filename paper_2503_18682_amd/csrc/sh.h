// Real spherical-harmonic colour shared by the preprocess kernel's colour
// phase and the colour backward (float32, contraction off, so both take the
// same clamp decision).
#pragma once

#include <hip/hip_runtime.h>

namespace rgs {

// Unit view direction camera centre -> mean as float32 (difference and norm
// in double, one reciprocal); *dist receives the distance.  Shared by the
// forward colour phase and the colour backward so both evaluate the same
// colour.
__device__ __forceinline__ void view_dir(const double (&m)[3], const double (&centre)[3], float (&dir)[3],
                                         double *dist)
{
#pragma clang fp contract(off)
    const double d0 = m[0] - centre[0], d1 = m[1] - centre[1], d2 = m[2] - centre[2];
    const double dn = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double inv = 1.0 / dn;
    dir[0] = (float)(d0 * inv);
    dir[1] = (float)(d1 * inv);
    dir[2] = (float)(d2 * inv);
    *dist = dn;
}

// Orthonormal real spherical harmonics up to degree 3 (index l^2 + l + m) in
// the sign convention of Gaussian-splatting colour models, evaluated in
// float32 (the colour is stored as float32).
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y)
{
#pragma clang fp contract(off)
    Y[0] = 0.28209479177387814f;
    if (DEG >= 1) {
        Y[1] = -0.48860251190291992f * y;
        Y[2] = 0.48860251190291992f * z;
        Y[3] = -0.48860251190291992f * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484305920792f * x * y;
        Y[5] = -1.0925484305920792f * y * z;
        Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
        Y[7] = -1.0925484305920792f * x * z;
        Y[8] = 0.54627421529603959f * (xx - yy);
    }
    if (DEG >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
        Y[10] = 2.8906114426405538f * x * y * z;
        Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
        Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
        Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
        Y[14] = 1.4453057213202769f * z * (xx - yy);
        Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
    }
}

// Unclamped colour 1/2 + sum_k Y_k c_k per channel (coefficients c[3 k + ch]).
template <int DEG>
__device__ __forceinline__ void sh_colour(const float *Y, const float *c, float *col)
{
#pragma clang fp contract(off)
    col[0] = col[1] = col[2] = 0.5f;
#pragma unroll
    for (int k = 0; k < (DEG + 1) * (DEG + 1); ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] += Y[k] * c[3 * k + ch];
}

// Direction gradient sum_k w_k dY_k / d(x, y, z) of a weighted basis (the
// basis gradients are formed and contracted on the fly).
template <int DEG>
__device__ __forceinline__ void sh_dir_grad(float x, float y, float z, const float *w, float *g)
{
    const float c1 = 0.48860251190291992f;
    const float c2a = 1.0925484305920792f, c2b = 0.31539156525252005f, c2c = 0.54627421529603959f;
    const float c3a = -0.59004358992664352f, c3b = 2.8906114426405538f, c3c = -0.45704579946446572f;
    const float c3d = 0.37317633259011540f, c3e = 1.4453057213202769f;
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
    if (DEG >= 1) {
        gy += -c1 * w[1];
        gz += c1 * w[2];
        gx += -c1 * w[3];
    }
    if (DEG >= 2) {
        gx += w[4] * (c2a * y);          gy += w[4] * (c2a * x);
        gy += w[5] * (-c2a * z);         gz += w[5] * (-c2a * y);
        gx += w[6] * (-2 * c2b * x);     gy += w[6] * (-2 * c2b * y); gz += w[6] * (4 * c2b * z);
        gx += w[7] * (-c2a * z);         gz += w[7] * (-c2a * x);
        gx += w[8] * (2 * c2c * x);      gy += w[8] * (-2 * c2c * y);
    }
    if (DEG >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx += w[9] * (6 * c3a * x * y);              gy += w[9] * (3 * c3a * (xx - yy));
        gx += w[10] * (c3b * y * z);                 gy += w[10] * (c3b * x * z);                 gz += w[10] * (c3b * x * y);
        gx += w[11] * (-2 * c3c * x * y);            gy += w[11] * (c3c * (4 * zz - xx - 3 * yy)); gz += w[11] * (8 * c3c * y * z);
        gx += w[12] * (-6 * c3d * x * z);            gy += w[12] * (-6 * c3d * y * z);            gz += w[12] * (3 * c3d * (2 * zz - xx - yy));
        gx += w[13] * (c3c * (4 * zz - 3 * xx - yy)); gy += w[13] * (-2 * c3c * x * y);           gz += w[13] * (8 * c3c * x * z);
        gx += w[14] * (2 * c3e * x * z);             gy += w[14] * (-2 * c3e * y * z);            gz += w[14] * (c3e * (xx - yy));
        gx += w[15] * (3 * c3a * (xx - yy));         gy += w[15] * (-6 * c3a * x * y);
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
}

}  // namespace rgs
