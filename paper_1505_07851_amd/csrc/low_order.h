// Low-order evaluations written out for the kernels of the lowest classes.  With the
// auxiliary R^(n) of the Hermite (McMurchie-Davidson) evaluation of the Eq. 5-6 integrals,
// R_000 = R^(0), R_{e_i} = X_i R^(1),
// R_{2 e_i} = X_i^2 R^(2) + R^(1) and R_{e_i + e_j} = X_i X_j R^(2) (i != j); the kernels
// contract these in factored form instead of forming every R_tuv first.
#pragma once
#include "pcm_internal.h"

// X_i = P_i - C_i in the kernel precision and R^(0) .. R^(N) of one (pair, point) evaluation
template <int N, typename T, typename B = T>
__device__ __forceinline__ void eval_Rn(double X, double Y, double Z, const PairHdr<T> &h, T zeta2, T zeta, T limk,
                                        const B *__restrict__ tab, T &x, T &y, T &z, T (&Rn)[N + 1]) {
    x = T(X);
    y = T(Y);
    z = T(Z);
    const T r2 = x * x + y * y + z * z;
    aux_Rn<N, T, B>(r2, h.p, h.limp, h.pf, h.pref, zeta2, zeta, limk, tab, Rn);
}
template <typename T, typename B = T>
__device__ __forceinline__ void eval_Rn1(double X, double Y, double Z, const PairHdr<T> &h, T zeta2, T zeta, T limk,
                                         const B *__restrict__ tab, T &x, T &y, T &z, T (&Rn)[2]) {
    eval_Rn<1, T, B>(X, Y, Z, h, zeta2, zeta, limk, tab, x, y, z, Rn);
}

// V_t += q R_t for every t with t + u + v <= 2 (index order of the Hermite tables: 000, 100,
// 010, 001, 200, 110, 101, 020, 011, 002), with q R^(1) and q R^(2) formed once
template <typename T>
__device__ __forceinline__ void acc_V2(double q, T x, T y, T z, const T (&Rn)[3], double (&V)[10]) {
    const double u1 = q * Rn[1], u2 = q * Rn[2];
    const double ux = u2 * x, uy = u2 * y, uz = u2 * z;
    V[0] = fma(q, Rn[0], V[0]);
    V[1] = fma(u1, x, V[1]);
    V[2] = fma(u1, y, V[2]);
    V[3] = fma(u1, z, V[3]);
    V[4] = fma(ux, x, V[4] + u1);
    V[5] = fma(ux, y, V[5]);
    V[6] = fma(ux, z, V[6]);
    V[7] = fma(uy, y, V[7] + u1);
    V[8] = fma(uy, z, V[8]);
    V[9] = fma(uz, z, V[9] + u1);
}

// V_t += q R_t for every t with t + u + v <= 3 (third-order entries in the order 300, 210, 201,
// 120, 111, 102, 030, 021, 012, 003): R_{3 e_i} = X_i^3 R^(3) + 3 X_i R^(2),
// R_{2 e_i + e_j} = X_i^2 X_j R^(3) + X_j R^(2), R_111 = X Y Z R^(3)
template <typename T>
__device__ __forceinline__ void acc_V3(double q, T x, T y, T z, const T (&Rn)[4], double (&V)[20]) {
    const double u1 = q * Rn[1], u2 = q * Rn[2], u3 = q * Rn[3];
    const double ux = u2 * x, uy = u2 * y, uz = u2 * z;
    V[0] = fma(q, Rn[0], V[0]);
    V[1] = fma(u1, x, V[1]);
    V[2] = fma(u1, y, V[2]);
    V[3] = fma(u1, z, V[3]);
    V[4] = fma(ux, x, V[4] + u1);
    V[5] = fma(ux, y, V[5]);
    V[6] = fma(ux, z, V[6]);
    V[7] = fma(uy, y, V[7] + u1);
    V[8] = fma(uy, z, V[8]);
    V[9] = fma(uz, z, V[9] + u1);
    const double wx = u3 * x, wy = u3 * y, wz = u3 * z;
    const double wxx = wx * x, wxy = wx * y, wyy = wy * y, wzz = wz * z;
    V[10] = fma(wxx, x, fma(3.0, ux, V[10]));
    V[11] = fma(wxx, y, V[11] + uy);
    V[12] = fma(wxx, z, V[12] + uz);
    V[13] = fma(wyy, x, V[13] + ux);
    V[14] = fma(wxy, z, V[14]);
    V[15] = fma(wzz, x, V[15] + ux);
    V[16] = fma(wyy, y, fma(3.0, uy, V[16]));
    V[17] = fma(wyy, z, V[17] + uz);
    V[18] = fma(wzz, y, V[18] + uy);
    V[19] = fma(wzz, z, fma(3.0, uz, V[19]));
}
