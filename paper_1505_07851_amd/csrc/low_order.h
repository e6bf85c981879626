// Order-1 evaluations written out for the FP64 kernels of the lowest classes.  With R^(0) and
// R^(1) of Sec. 4a's Hermite scheme, R_000 = R^(0) and R_{e_i} = X_i R^(1); the contractions
// below factor R^(1) out of the three first-order terms, which saves two multiplications per
// (pair, point) evaluation against forming R_tuv first.
#pragma once
#include "pcm_internal.h"

// X_i = P_i - C_i in the kernel precision and R^(0), R^(1) of one (pair, point) evaluation
template <typename T>
__device__ __forceinline__ void eval_Rn1(double X, double Y, double Z, const PairHdr<T> &h, T zeta2, T zeta, T limk,
                                         const T *__restrict__ tab, T &x, T &y, T &z, T (&Rn)[2]) {
    x = T(X);
    y = T(Y);
    z = T(Z);
    const T r2 = x * x + y * y + z * z;
    aux_Rn<1, T>(r2, h.p, h.limp, h.pf, h.pref, zeta2, zeta, limk, tab, Rn);
}
