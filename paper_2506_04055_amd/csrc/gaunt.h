// Couplings of the real spherical harmonics of sh.h (degree <= 3) as
// constant expressions, and a compile-time loop.
//
// G(i, j, k) = (1 / 4 pi) int Y_i Y_j Y_k dOmega over harmonic slots
// i = l^2 + m, evaluated by a product rule: 8-point Gauss-Legendre in
// cos(theta) times 16 uniform points in phi.  The integrand is a polynomial of
// degree at most 9 on the sphere; the rule integrates cos(theta) polynomials
// to degree 15 and trigonometric polynomials in phi to degree 15 exactly, so
// the values are exact up to rounding.  Everything here is constexpr (the
// trigonometric values by series, square roots by Newton's method) so that
// kernels can unroll over the nonzero couplings only.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sh.h"

namespace mlp {
namespace cg {

constexpr double kPi = 3.14159265358979323846;

constexpr double csqrt(double x) {
    if (x <= 0.0) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 200; i++) r = 0.5 * (r + x / r);
    return r;
}

constexpr double ccos(double x) {
    while (x > kPi) x -= 2.0 * kPi;
    while (x < -kPi) x += 2.0 * kPi;
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 30; k++) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}

constexpr double csin(double x) { return ccos(x - 0.5 * kPi); }

// P_n(z) and P_n'(z) by the three-term recurrence
constexpr void legendre(int n, double z, double &p, double &dp) {
    double p1 = 1.0, p2 = 0.0;
    for (int j = 1; j <= n; j++) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
    }
    p = p1;
    dp = n * (z * p1 - p2) / (z * z - 1.0);
}

constexpr int NZ = 8, NPHI = 16, NQ = NZ * NPHI;

struct Quad {
    double Y[NQ][16] = {};
    double w[NQ] = {};
};

constexpr Quad make_quad() {
    Quad Q{};
    for (int i = 0; i < NZ; i++) {
        double z = ccos(kPi * (i + 0.75) / (NZ + 0.5)), p = 0.0, dp = 0.0;
        for (int it = 0; it < 60; it++) {
            legendre(NZ, z, p, dp);
            z -= p / dp;
        }
        legendre(NZ, z, p, dp);
        const double wz = 2.0 / ((1.0 - z * z) * dp * dp), s = csqrt(1.0 - z * z);
        for (int b = 0; b < NPHI; b++) {
            const double ph = 2.0 * kPi * b / NPHI;
            sh16<double>(s * ccos(ph), s * csin(ph), z, Q.Y[i * NPHI + b]);
            Q.w[i * NPHI + b] = wz / (2.0 * NPHI);   // (2 pi / NPHI) / (4 pi)
        }
    }
    return Q;
}

struct Table {
    double g[16][16][16] = {};
};

constexpr Table make_table() {
    const Quad Q = make_quad();
    Table T{};
    for (int i = 0; i < 16; i++)
        for (int j = 0; j < 16; j++)
            for (int k = 0; k < 16; k++) {
                double s = 0.0;
                for (int q = 0; q < NQ; q++) s += Q.w[q] * Q.Y[q][i] * Q.Y[q][j] * Q.Y[q][k];
                // couplings that vanish by symmetry come out at rounding level
                T.g[i][j][k] = (s > 1e-12 || s < -1e-12) ? s : 0.0;
            }
    return T;
}

inline constexpr Table kG = make_table();

// G(l1, l2, L)[a][b][c]
constexpr double coupling(int l1, int a, int l2, int b, int L, int c) { return kG.g[l1 * l1 + a][l2 * l2 + b][L * L + c]; }

// degrees l1 x l2 -> L that a coupling keeps: the triangle rule and even
// l1 + l2 + L (every feature keeps the parity of its degree)
constexpr bool couples(int l1, int l2, int L) {
    const int d = l1 > l2 ? l1 - l2 : l2 - l1;
    return d <= L && L <= l1 + l2 && (l1 + l2 + L) % 2 == 0;
}

// ---------------------------------------------------------------------------
// Compile-time loop: sfor<N>(f) calls f(std::integral_constant<int, I>) for
// I = 0 .. N-1, so that I is usable in constant expressions in f.
// ---------------------------------------------------------------------------
template <int... I> struct iseq {};
template <int N, int... I> struct make_iseq : make_iseq<N - 1, N - 1, I...> {};
template <int... I> struct make_iseq<0, I...> {
    using type = iseq<I...>;
};
template <class F, int... I>
__host__ __device__ __forceinline__ void sfor_impl(F &f, iseq<I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, typename make_iseq<N>::type{});
}

}  // namespace cg
}  // namespace mlp
