// Real spherical harmonics of degree <= 3 (component normalisation,
// sum_m Y_lm^2 = 2l + 1) in Cartesian form, their gradient, and the
// polynomial cutoff envelope; host and device (the host builds coupling
// tables from the same harmonics the kernels evaluate).
#pragma once
#include <hip/hip_runtime.h>

namespace mlp {

// ---------------------------------------------------------------------------
// Spherical harmonics, component normalisation, degree <= 3, as polynomials
// of the unit vector (x, y, z), and the tangential gradient of sum_m g_m Y_m.
// ---------------------------------------------------------------------------
template <class T>
__host__ __device__ constexpr inline void sh16(T x, T y, T z, T *Y) {
    const T s3 = (T)1.7320508075688772, s15 = (T)3.872983346207417, s5 = (T)2.23606797749979;
    const T s70 = (T)8.366600265340756, s105 = (T)10.246950765959598, s42 = (T)6.48074069840786,
            s7 = (T)2.6457513110645907;
    Y[0] = (T)1;
    Y[1] = s3 * y;
    Y[2] = s3 * z;
    Y[3] = s3 * x;
    Y[4] = s15 * x * y;
    Y[5] = s15 * y * z;
    Y[6] = (T)0.5 * s5 * ((T)3 * z * z - (T)1);
    Y[7] = s15 * x * z;
    Y[8] = (T)0.5 * s15 * (x * x - y * y);
    Y[9] = (T)0.25 * s70 * y * ((T)3 * x * x - y * y);
    Y[10] = s105 * x * y * z;
    Y[11] = (T)0.25 * s42 * y * ((T)5 * z * z - (T)1);
    Y[12] = (T)0.5 * s7 * z * ((T)5 * z * z - (T)3);
    Y[13] = (T)0.25 * s42 * x * ((T)5 * z * z - (T)1);
    Y[14] = (T)0.5 * s105 * z * (x * x - y * y);
    Y[15] = (T)0.25 * s70 * x * (x * x - (T)3 * y * y);
}

// sum_m g[m] grad Y_m, the gradient of the polynomial forms above (the
// caller projects it onto the tangent plane)
__host__ __device__ inline void sh16_grad(float x, float y, float z, const float *g, float &ox, float &oy,
                                          float &oz) {
    const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s5 = 2.23606797749979f;
    const float s70 = 8.366600265340756f, s105 = 10.246950765959598f, s42 = 6.48074069840786f,
                s7 = 2.6457513110645907f;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    gx += s3 * g[3];
    gy += s3 * g[1];
    gz += s3 * g[2];
    gx += s15 * (g[4] * y + g[7] * z + g[8] * x);
    gy += s15 * (g[4] * x + g[5] * z - g[8] * y);
    gz += s15 * (g[5] * y + g[7] * x) + 3.f * s5 * z * g[6];
    const float a9 = 0.25f * s70 * g[9], a15 = 0.25f * s70 * g[15];
    gx += a9 * 6.f * x * y + a15 * (3.f * x * x - 3.f * y * y);
    gy += a9 * (3.f * x * x - 3.f * y * y) - a15 * 6.f * x * y;
    gx += s105 * g[10] * y * z;
    gy += s105 * g[10] * x * z;
    gz += s105 * g[10] * x * y;
    const float a11 = 0.25f * s42 * g[11], a13 = 0.25f * s42 * g[13];
    gy += a11 * (5.f * z * z - 1.f);
    gz += a11 * 10.f * y * z + a13 * 10.f * x * z;
    gx += a13 * (5.f * z * z - 1.f);
    gz += 0.5f * s7 * g[12] * (15.f * z * z - 3.f);
    const float a14 = 0.5f * s105 * g[14];
    gx += a14 * 2.f * x * z;
    gy -= a14 * 2.f * y * z;
    gz += a14 * (x * x - y * y);
    ox = gx;
    oy = gy;
    oz = gz;
}

// Envelope u(x) and du/dx for order p.
__host__ __device__ inline void envelope(float x, int p, float &u, float &du) {
    const float a = 0.5f * (p + 1) * (p + 2), b = (float)(p * (p + 2)), c = 0.5f * p * (p + 1);
    float xp1 = 1.f;  // x^(p-1)
    for (int q = 1; q < p; q++) xp1 *= x;
    const float xp = xp1 * x;
    u = 1.f - a * xp + b * xp * x - c * xp * x * x;
    du = -a * p * xp1 + b * (p + 1) * xp - c * (p + 2) * xp * x;
}

}  // namespace mlp
