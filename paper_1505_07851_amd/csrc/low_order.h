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

// Far-field factored sums of the pair-per-lane kernels (FP64 records).  In the far field
// R^(n) = pf (-1)^n (2n-1)!! / r^(2n+1), so with s_n = q (-1)^n R^(n) / ((2n-1)!! pf) = q / r^(2n+1)
// the V_tuv of acc_V2 / acc_V3 are pf times fixed combinations of
//   S0 = sum s0, S1 = sum s1, S1_i = sum s1 X_i, S2_i = sum s2 X_i, S2_ij = sum s2 X_i X_j,
//   S3_ijk = sum s3 X_i X_j X_k,
// e.g. V_200 = pf (3 S2_xx - S1) and V_300 = pf (9 S2_x - 15 S3_xxx).  A far evaluation then
// steps s_n = s_(n-1) / r^2 instead of forming R^(n) and multiplying each by q; a near one enters
// the same sums with s_n = q R^(n) (-1)^n / ((2n-1)!! pf).  pf is applied once per item.
// Sum layout (N = 1, 5 sums): S0, S1, S1_x, S1_y, S1_z (S1 unused at this order);
// N = 2 adds (11 sums): S2_xx, S2_xy, S2_xz, S2_yy, S2_yz, S2_zz;
// N = 3 adds (24 sums): S2_x, S2_y, S2_z, S3_xxx, S3_xxy, S3_xxz, S3_xyy, S3_xyz, S3_xzz, S3_yyy,
// S3_yyz, S3_yzz, S3_zzz;
// N = 4 adds (46 sums): S2, S3_xx, S3_xy, S3_xz, S3_yy, S3_yz, S3_zz, then S4 over the quartic
// monomials xxxx, xxxy, xxxz, xxyy, xxyz, xxzz, xyyy, xyyz, xyzz, xzzz, yyyy, yyyz, yyzz, yzzz, zzzz.
template <int N> __host__ __device__ constexpr int nsums() { return N == 1 ? 5 : (N == 2 ? 11 : (N == 3 ? 24 : 46)); }
template <int N> __host__ __device__ constexpr int nvsum() { return N == 1 ? 4 : (N == 2 ? 10 : (N == 3 ? 20 : 35)); }

// s_0 .. s_N of one (pair, point) evaluation; (X, Y, Z) = P - C, ipf = 1 / pf (far_scale)
template <int N, typename B>
__device__ __forceinline__ void eval_s(double X, double Y, double Z, const PairHdr<double> &h, double ipf,
                                       double zeta2, double zeta, double limk, const B *__restrict__ tab, double q,
                                       double &x, double &y, double &z, double (&s)[N + 1]) {
    x = X;
    y = Y;
    z = Z;
    const double r2 = x * x + y * y + z * z;
    if (r2 >= h.limp + limk) {
        const double ri = rsq_fast(r2), ri2 = ri * ri;
        s[0] = q * ri;
#pragma unroll
        for (int n = 1; n <= N; ++n) s[n] = s[n - 1] * ri2;
    } else {
        double Rn[N + 1];
        aux_Rn_near<N, double, B>(r2, h.p, h.pref, zeta2, zeta, tab, Rn);
        constexpr double c[5] = {1.0, -1.0, 1.0 / 3.0, -1.0 / 15.0, 1.0 / 105.0};  // (-1)^n / (2n-1)!!
        const double qi = q * ipf;
#pragma unroll
        for (int n = 0; n <= N; ++n) s[n] = (qi * Rn[n]) * c[n];
    }
}

// 1 / pf of a pair (zero for a pair whose prefactor vanished)
__device__ __forceinline__ double far_scale(double pf) { return pf != 0.0 ? 1.0 / pf : 0.0; }

template <int N>
__device__ __forceinline__ void acc_S(const double (&s)[N + 1], double x, double y, double z,
                                      double (&S)[nsums<N>()]) {
    S[0] += s[0];
    S[2] = fma(s[1], x, S[2]);
    S[3] = fma(s[1], y, S[3]);
    S[4] = fma(s[1], z, S[4]);
    if constexpr (N >= 2) {
        S[1] += s[1];
        const double ax = s[2] * x, ay = s[2] * y, az = s[2] * z;
        S[5] = fma(ax, x, S[5]);
        S[6] = fma(ax, y, S[6]);
        S[7] = fma(ax, z, S[7]);
        S[8] = fma(ay, y, S[8]);
        S[9] = fma(ay, z, S[9]);
        S[10] = fma(az, z, S[10]);
        if constexpr (N >= 3) {
            S[11] += ax;
            S[12] += ay;
            S[13] += az;
            const double bx = s[3] * x, by = s[3] * y, bz = s[3] * z;
            const double bxx = bx * x, bxy = bx * y, byy = by * y, bzz = bz * z;
            S[14] = fma(bxx, x, S[14]);
            S[15] = fma(bxx, y, S[15]);
            S[16] = fma(bxx, z, S[16]);
            S[17] = fma(byy, x, S[17]);
            S[18] = fma(bxy, z, S[18]);
            S[19] = fma(bzz, x, S[19]);
            S[20] = fma(byy, y, S[20]);
            S[21] = fma(byy, z, S[21]);
            S[22] = fma(bzz, y, S[22]);
            S[23] = fma(bzz, z, S[23]);
            if constexpr (N == 4) {
                S[24] += s[2];
                S[25] += bxx;
                S[26] += bxy;
                S[27] = fma(bx, z, S[27]);
                S[28] += byy;
                S[29] = fma(by, z, S[29]);
                S[30] += bzz;
                const double cx = s[4] * x, cy = s[4] * y, cz = s[4] * z;
                const double cxx = cx * x, cxy = cx * y, cyy = cy * y, czz = cz * z;
                const double cxxx = cxx * x, cxyy = cyy * x, cxzz = czz * x, cxyz = cxy * z;
                const double cyyy = cyy * y, cyzz = czz * y, czzz = czz * z;
                S[31] = fma(cxxx, x, S[31]);  // xxxx
                S[32] = fma(cxxx, y, S[32]);  // xxxy
                S[33] = fma(cxxx, z, S[33]);  // xxxz
                S[34] = fma(cxyy, x, S[34]);  // xxyy
                S[35] = fma(cxyz, x, S[35]);  // xxyz
                S[36] = fma(cxzz, x, S[36]);  // xxzz
                S[37] = fma(cxyy, y, S[37]);  // xyyy
                S[38] = fma(cxyy, z, S[38]);  // xyyz
                S[39] = fma(cxzz, y, S[39]);  // xyzz
                S[40] = fma(cxzz, z, S[40]);  // xzzz
                S[41] = fma(cyyy, y, S[41]);  // yyyy
                S[42] = fma(cyyy, z, S[42]);  // yyyz
                S[43] = fma(cyzz, y, S[43]);  // yyzz
                S[44] = fma(cyzz, z, S[44]);  // yzzz
                S[45] = fma(czzz, z, S[45]);  // zzzz
            }
        }
    }
}

// V_tuv (the index order of acc_V2 / acc_V3) from the sums
template <int N>
__device__ __forceinline__ void fin_S(double pf, const double (&S)[nsums<N>()], double (&V)[nvsum<N>()]) {
    V[0] = pf * S[0];
    V[1] = -pf * S[2];
    V[2] = -pf * S[3];
    V[3] = -pf * S[4];
    if constexpr (N >= 2) {
        const double p3 = 3.0 * pf;
        V[4] = pf * fma(3.0, S[5], -S[1]);
        V[5] = p3 * S[6];
        V[6] = p3 * S[7];
        V[7] = pf * fma(3.0, S[8], -S[1]);
        V[8] = p3 * S[9];
        V[9] = pf * fma(3.0, S[10], -S[1]);
        if constexpr (N >= 3) {
            V[10] = pf * fma(-15.0, S[14], 9.0 * S[11]);
            V[11] = pf * fma(-15.0, S[15], 3.0 * S[12]);
            V[12] = pf * fma(-15.0, S[16], 3.0 * S[13]);
            V[13] = pf * fma(-15.0, S[17], 3.0 * S[11]);
            V[14] = -15.0 * pf * S[18];
            V[15] = pf * fma(-15.0, S[19], 3.0 * S[11]);
            V[16] = pf * fma(-15.0, S[20], 9.0 * S[12]);
            V[17] = pf * fma(-15.0, S[21], 3.0 * S[13]);
            V[18] = pf * fma(-15.0, S[22], 3.0 * S[12]);
            V[19] = pf * fma(-15.0, S[23], 9.0 * S[13]);
            if constexpr (N == 4) {
                // order 4: R_400 = X^4 R4 + 6 X^2 R3 + 3 R2, R_310 = X^3 Y R4 + 3 X Y R3,
                // R_220 = X^2 Y^2 R4 + (X^2 + Y^2) R3 + R2, R_211 = X^2 Y Z R4 + Y Z R3, with
                // R^(n) = pf (-1)^n (2n-1)!! s_n / q: the constants 105, -15 and 3
                const double s2 = 3.0 * S[24];
                V[20] = pf * fma(105.0, S[31], fma(-90.0, S[25], 3.0 * s2));  // 400
                V[21] = pf * fma(105.0, S[32], -45.0 * S[26]);               // 310
                V[22] = pf * fma(105.0, S[33], -45.0 * S[27]);               // 301
                V[23] = pf * fma(105.0, S[34], fma(-15.0, S[25] + S[28], s2)); // 220
                V[24] = pf * fma(105.0, S[35], -15.0 * S[29]);               // 211
                V[25] = pf * fma(105.0, S[36], fma(-15.0, S[25] + S[30], s2)); // 202
                V[26] = pf * fma(105.0, S[37], -45.0 * S[26]);               // 130
                V[27] = pf * fma(105.0, S[38], -15.0 * S[27]);               // 121
                V[28] = pf * fma(105.0, S[39], -15.0 * S[26]);               // 112
                V[29] = pf * fma(105.0, S[40], -45.0 * S[27]);               // 103
                V[30] = pf * fma(105.0, S[41], fma(-90.0, S[28], 3.0 * s2));  // 040
                V[31] = pf * fma(105.0, S[42], -45.0 * S[29]);               // 031
                V[32] = pf * fma(105.0, S[43], fma(-15.0, S[28] + S[30], s2)); // 022
                V[33] = pf * fma(105.0, S[44], -45.0 * S[29]);               // 013
                V[34] = pf * fma(105.0, S[45], fma(-90.0, S[30], 3.0 * s2));  // 004
            }
        }
    }
}
