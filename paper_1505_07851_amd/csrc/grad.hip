// Gradient of the solvation energy at fixed density (Sec. 2, Eq. 14; Sec. 4c, Eq. 22):
//
//   dE = z^T (dB^T) q + (d* c^T) q + 1/(2f) q^T (dA) q
//
// Outputs: g_nuc[I] = dE/dR_I with the surface points held fixed (basis centres, nuclear
// positions in B, the R_J inside the switching functions of A_kk) and g_surf[k] = dE/dr_k.
//
// The c term follows Eq. 22: per primitive pair, ga/gb (basis-centre derivatives) are
// reductions over points and gc (operator-centre derivative) is a reduction over pairs.
//   ga, gb:  V'_tuv = sum_k q_k R_tuv up to L+1 (lane = pair), then per pair
//            dA [a|J|b] = 2a [a+1|J|b] - a_x [a-1|J|b] contracted with -w P c c;
//   gc:      dC R_tuv = -R_{t+1,u,v}: lane = point, contracted with the esp coefficients.
// Per-atom sums run over fixed per-atom lists, so every result is bitwise reproducible.
#include "pcm_internal.h"
#include "low_order.h"
#include "contract.h"

#include <array>
#include <cstring>

// -------------------------------------------------------------------------------------------
// gc: g_surf contribution of the c term, partial over a chunk of pairs (3 rows per chunk)
// -------------------------------------------------------------------------------------------
// Work of one molecule and class in a (possibly batched) launch; items are numbered from `base`.
struct GradPtsDesc {
    const unsigned char *rec;  // class records (header + D_tuv), padded to REC_PAD
    const void *pts;           // PtInt<T> [Mpad]
    const int *pperm;          // point taken by each lane (null: surface order)
    double *part;              // partial rows [row][3][M]
    long long base;            // first item: (point tile, pair chunk), tile fastest
    int stride, n_pad, chunk, M, ntile, row0;
};
struct GradVDesc {
    const unsigned char *rec;  // class records
    const int *perm;           // record taken by each lane, class-local (null: list order)
    const void *pts;           // PtInt<T> [Mpad]
    const double *q;           // charges, zero past M [Mpad]
    double *vout;              // [chunk][tuv][pair]
    long long base;            // first item: (pair tile, point chunk), tile fastest
    int stride, n_pairs, Mpad, chunk, nptile;
};

// WC: also accumulate the potential c_k = sum_t D_t R_t (Eqs. 5-6), which the R^(n) of the
// derivative contain (orders 0 .. L of the L+1 evaluated); rows are then 4 wide (gx, gy, gz, c)
template <int L, typename T, typename B, bool WC>
__global__ __launch_bounds__(256) void k_grad_pts(const GradPtsDesc *__restrict__ ds, int nd, long long n_items,
                                                  const B *__restrict__ boys_g) {
    // PF: the records of the next batch are requested before the current batch is evaluated and
    // waited for after it, so the scalar-load latency overlaps the evaluation
    constexpr bool PF = L <= 2;
    constexpr int NT = ntuv(L), PB = PF ? pair_batch_pf<L>() : pair_batch<L + 1>();
    __shared__ B tab[boys_lds_size<B, L + 1>()];
    load_boys<B, L + 1>(tab, boys_g);
    {  // one item per block (the grid covers every item; a loop over items costs registers here)
        const long long it = blockIdx.x;
        if (it >= n_items) return;
        const GradPtsDesc &d = ds[find_desc(ds, nd, it)];
        const long long local = it - d.base;
        const int tile = (int)(local % d.ntile), ch = (int)(local / d.ntile);
        const cptr<unsigned char> rec = as_const(d.rec);
        const PtInt<T> *__restrict__ pts = reinterpret_cast<const PtInt<T> *>(d.pts);
        const int M = d.M, stride = d.stride;
        const int k = tile * 256 + threadIdx.x;
        const int kk = k < M ? (d.pperm ? d.pperm[k] : k) : M - 1;
        const PtInt<T> me = pts[kk];
        const int p0 = ch * d.chunk;
        const int p1 = min(d.n_pad, p0 + d.chunk);
        double gx = 0.0, gy = 0.0, gz = 0.0, cc = 0.0;
        auto load = [&](int i0, PairHdr<T>(&hh)[PB], T(&DD)[PB][NT]) {
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const cptr<unsigned char> r = rec + (size_t)(i0 + b) * stride;
                hh[b] = *(cptr<PairHdr<T>>)(r);
                const cptr<T> dd = (cptr<T>)(r + sizeof(PairHdr<T>));
#pragma unroll
                for (int t = 0; t < NT; ++t) DD[b][t] = dd[t];
            }
        };
        PairHdr<T> h[PB];
        T D[PB][NT];
        if constexpr (PF) load(p0, h, D);
        for (int ip = p0; ip < p1; ip += PB) {
            PairHdr<T> hn[PB];
            T Dn[PB][NT];
            if constexpr (PF)
                load(ip + PB < p1 ? ip + PB : ip, hn, Dn);  // the last batch re-reads itself
            else
                load(ip, h, D);
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                if constexpr (L == 3) {
                    // g_i = d/dX_i of S = D_0 R^(0) + lin R^(1) + quad R^(2) + C R^(3) (the L = 3
                    // potential; quad holds the second-order terms and the first-order parts of the
                    // third-order R_tuv, C the cubic form): g_i = X_i (D_0 R^(1) + lin R^(2) + quad R^(3)
                    //   + C R^(4)) + D_{e_i} R^(1) + (d quad/dX_i) R^(2) + (dC/dX_i) R^(3),
                    // with C = (X dC/dX + Y dC/dY + Z dC/dZ) / 3 (C is homogeneous of degree 3)
                    const T *Db = D[b];
                    T x, y, z, Rn[5];
                    eval_Rn<4, T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim,
                                  tab, x, y, z, Rn);
                    const T xx = x * x, xy = x * y, xz = x * z, yy = y * y, yz = y * z, zz = z * z;
                    const T two = T(2), three = T(3);
                    // D index: 10 300, 11 210, 12 201, 13 120, 14 111, 15 102, 16 030, 17 021, 18 012, 19 003
                    const T dcx = fma(three * Db[10], xx, fma(two * Db[11], xy, fma(two * Db[12], xz,
                                  fma(Db[13], yy, fma(Db[14], yz, Db[15] * zz)))));
                    const T dcy = fma(Db[11], xx, fma(two * Db[13], xy, fma(Db[14], xz,
                                  fma(three * Db[16], yy, fma(two * Db[17], yz, Db[18] * zz)))));
                    const T dcz = fma(Db[12], xx, fma(Db[14], xy, fma(two * Db[15], xz,
                                  fma(Db[17], yy, fma(two * Db[18], yz, three * Db[19] * zz)))));
                    const T cub = fma(x, dcx, fma(y, dcy, z * dcz)) * (T(1) / three);
                    const T gqx = fma(two * Db[4], x, fma(Db[5], y, Db[6] * z));
                    const T gqy = fma(Db[5], x, fma(two * Db[7], y, Db[8] * z));
                    const T gqz = fma(Db[6], x, fma(Db[8], y, two * Db[9] * z));
                    const T bx = fma(three, Db[10], Db[13] + Db[15]);
                    const T by = fma(three, Db[16], Db[11] + Db[18]);
                    const T bz = fma(three, Db[19], Db[12] + Db[17]);
                    const T quad = fma(T(0.5), fma(x, gqx, fma(y, gqy, z * gqz)), fma(bx, x, fma(by, y, bz * z)));
                    const T lin = fma(Db[1], x, fma(Db[2], y, fma(Db[3], z, Db[4] + Db[7] + Db[9])));
                    const T a = fma(cub, Rn[4], fma(quad, Rn[3], fma(lin, Rn[2], Db[0] * Rn[1])));
                    const T ex = fma(dcx, Rn[3], fma(gqx + bx, Rn[2], Db[1] * Rn[1]));
                    const T ey = fma(dcy, Rn[3], fma(gqy + by, Rn[2], Db[2] * Rn[1]));
                    const T ez = fma(dcz, Rn[3], fma(gqz + bz, Rn[2], Db[3] * Rn[1]));
                    if constexpr (sizeof(T) == 8) {
                        gx = fma(a, x, gx + ex);
                        gy = fma(a, y, gy + ey);
                        gz = fma(a, z, gz + ez);
                        if constexpr (WC) {
                            cc = fma(Db[0], Rn[0], cc);
                            cc = fma(lin, Rn[1], cc);
                            cc = fma(quad, Rn[2], cc);
                            cc = fma(cub, Rn[3], cc);
                        }
                    } else {
                        gx += (double)fma(a, x, ex);
                        gy += (double)fma(a, y, ey);
                        gz += (double)fma(a, z, ez);
                        if constexpr (WC) cc += (double)fma(cub, Rn[3], fma(quad, Rn[2], fma(lin, Rn[1], Db[0] * Rn[0])));
                    }
                    continue;
                }
                if constexpr (L == 2) {
                    // g_i = d/dX_i of S = D_0 R^(0) + lin R^(1) + Q R^(2) (the L = 2 potential, with
                    // d R^(n) / dX_i = X_i R^(n+1)): g_i = X_i (D_0 R^(1) + lin R^(2) + Q R^(3))
                    //   + D_{e_i} R^(1) + (dQ/dX_i) R^(2)
                    const T *Db = D[b];
                    T x, y, z, Rn[4];
                    eval_Rn<3, T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim,
                                  tab, x, y, z, Rn);
                    const T q1 = fma(Db[4], x, fma(Db[5], y, Db[6] * z));  // D_200 X + D_110 Y + D_101 Z
                    const T q2 = fma(Db[7], y, Db[8] * z);                 // D_020 Y + D_011 Z
                    const T zz = Db[9] * z;                                // D_002 Z
                    const T qf = fma(x, q1, fma(y, q2, z * zz));
                    const T lin = fma(Db[1], x, fma(Db[2], y, fma(Db[3], z, Db[4] + Db[7] + Db[9])));
                    const T a = fma(qf, Rn[3], fma(lin, Rn[2], Db[0] * Rn[1]));
                    const T gqx = fma(Db[4], x, q1);
                    const T gqy = fma(Db[5], x, fma(Db[7], y, q2));
                    const T gqz = fma(Db[6], x, fma(Db[8], y, zz + zz));
                    if constexpr (sizeof(T) == 8) {
                        gx = fma(a, x, fma(Db[1], Rn[1], fma(gqx, Rn[2], gx)));
                        gy = fma(a, y, fma(Db[2], Rn[1], fma(gqy, Rn[2], gy)));
                        gz = fma(a, z, fma(Db[3], Rn[1], fma(gqz, Rn[2], gz)));
                        if constexpr (WC) {
                            cc = fma(Db[0], Rn[0], cc);
                            cc = fma(lin, Rn[1], cc);
                            cc = fma(qf, Rn[2], cc);
                        }
                    } else {  // FP32 evaluation, one FP64 add per pair and component
                        gx += (double)fma(a, x, fma(Db[1], Rn[1], gqx * Rn[2]));
                        gy += (double)fma(a, y, fma(Db[2], Rn[1], gqy * Rn[2]));
                        gz += (double)fma(a, z, fma(Db[3], Rn[1], gqz * Rn[2]));
                        if constexpr (WC) cc += (double)fma(qf, Rn[2], fma(lin, Rn[1], Db[0] * Rn[0]));
                    }
                    continue;
                }
                if constexpr (L == 1) {
                    // g_i = sum_t D_t R_{t + e_i} = X_i (D_0 R^(1) + R^(2) w) + D_{e_i} R^(1),
                    // w = D_100 X + D_010 Y + D_001 Z
                    T x, y, z, Rn[3];
                    eval_Rn<2, T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim,
                                  tab, x, y, z, Rn);
                    const T w = fma(D[b][1], x, fma(D[b][2], y, D[b][3] * z));
                    const T a = fma(Rn[2], w, D[b][0] * Rn[1]);
                    if constexpr (sizeof(T) == 8) {
                        gx = fma(a, x, fma(D[b][1], Rn[1], gx));
                        gy = fma(a, y, fma(D[b][2], Rn[1], gy));
                        gz = fma(a, z, fma(D[b][3], Rn[1], gz));
                        if constexpr (WC) {
                            cc = fma(D[b][0], Rn[0], cc);
                            cc = fma(w, Rn[1], cc);
                        }
                    } else {
                        gx += (double)fma(a, x, D[b][1] * Rn[1]);
                        gy += (double)fma(a, y, D[b][2] * Rn[1]);
                        gz += (double)fma(a, z, D[b][3] * Rn[1]);
                        if constexpr (WC) cc += (double)fma(w, Rn[1], D[b][0] * Rn[0]);
                    }
                    continue;
                }
                if constexpr (L == 0) {  // D R_{e_i} = (D R^(1)) X_i
                    T x, y, z, Rn[2];
                    eval_Rn1<T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim, tab,
                                x, y, z, Rn);
                    const T t1 = D[b][0] * Rn[1];
                    if constexpr (sizeof(T) == 8) {
                        gx = fma(t1, x, gx);
                        gy = fma(t1, y, gy);
                        gz = fma(t1, z, gz);
                        if constexpr (WC) cc = fma(D[b][0], Rn[0], cc);
                    } else {
                        gx += (double)(t1 * x);
                        gy += (double)(t1 * y);
                        gz += (double)(t1 * z);
                        if constexpr (WC) cc += (double)(D[b][0] * Rn[0]);
                    }
                    continue;
                }
                T R[ntuv(L + 1)];
                eval_R<L + 1, T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim, tab,
                                 R);
                if constexpr (sizeof(T) == 8) {  // FP64: straight into the accumulators
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        gx = fma(D[b][t], R[TuvShift<L>::x(t)], gx);
                        gy = fma(D[b][t], R[TuvShift<L>::y(t)], gy);
                        gz = fma(D[b][t], R[TuvShift<L>::z(t)], gz);
                        if constexpr (WC) cc = fma(D[b][t], R[t], cc);  // orders <= L come first in R
                    }
                } else {  // FP32 evaluation, one FP64 add per pair
                    T sx = T(0), sy = T(0), sz = T(0), sc = T(0);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        sx = fma(D[b][t], R[TuvShift<L>::x(t)], sx);
                        sy = fma(D[b][t], R[TuvShift<L>::y(t)], sy);
                        sz = fma(D[b][t], R[TuvShift<L>::z(t)], sz);
                        if constexpr (WC) sc = fma(D[b][t], R[t], sc);
                    }
                    gx += (double)sx;
                    gy += (double)sy;
                    gz += (double)sz;
                    if constexpr (WC) cc += (double)sc;
                }
            }
            if constexpr (PF) {
                // the next batch's records are needed only here, after this batch's evaluation
                // (the empty statements order the wait after the accumulations)
                asm volatile("" ::"v"(gx), "v"(gy), "v"(gz), "v"(cc));
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    pin_sgpr(hn[b]);
#pragma unroll
                    for (int t = 0; t < NT; ++t) pin_sgpr(Dn[b][t]);
                    h[b] = hn[b];
#pragma unroll
                    for (int t = 0; t < NT; ++t) D[b][t] = Dn[b][t];
                }
            }
        }
        if (k < M) {
            const size_t base = (size_t)(d.row0 + ch) * (WC ? 4 : 3) * M;
            d.part[base + kk] = gx;
            d.part[base + M + kk] = gy;
            d.part[base + 2 * M + kk] = gz;
            if constexpr (WC) d.part[base + 3 * M + kk] = cc;
        }
    }
}

// -------------------------------------------------------------------------------------------
// V'_tuv up to L+1 per pair (lane = pair), weights q_k; same as the Fock accumulation
// -------------------------------------------------------------------------------------------
template <int L, typename T, typename B>
__global__ __launch_bounds__(256, L == 3 ? 3 : 1) void k_grad_v(const GradVDesc *__restrict__ ds, int nd, long long n_items,
                                                const B *__restrict__ boys_g) {
    __shared__ B tab[boys_lds_size<B, L + 1>()];
    load_boys<B, L + 1>(tab, boys_g);
    constexpr int NT = ntuv(L + 1);
    // points per batch: fewer for the larger V' sets so that more waves stay resident
    constexpr int PB = L <= 1 ? PT_BATCH : (L == 2 && sizeof(T) == 4 ? 2 : 1);
    {  // one item per block, as in k_grad_pts
        const long long it = blockIdx.x;
        if (it >= n_items) return;
        const GradVDesc &d = ds[find_desc(ds, nd, it)];
        const long long local = it - d.base;
        const int ptile = (int)(local % d.nptile), ch = (int)(local / d.nptile);
        const int n_pairs = d.n_pairs;
        const int ip = ptile * 256 + threadIdx.x;
        const int ipp = d.perm ? d.perm[ip < n_pairs ? ip : n_pairs - 1] : (ip < n_pairs ? ip : n_pairs - 1);
        const PairHdr<T> h = *reinterpret_cast<const PairHdr<T> *>(d.rec + (size_t)ipp * d.stride);
        const cptr<PtInt<T>> pts = as_const(reinterpret_cast<const PtInt<T> *>(d.pts));
        const cptr<double> q = as_const(d.q);
        const int k0 = ch * d.chunk;
        const int k1 = min(d.Mpad, k0 + d.chunk);
        double V[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) V[t] = 0.0;
        // FP64 records (V' up to order 1 .. 4): the far-field factored sums of low_order.h
        constexpr bool FS = sizeof(T) == 8 && L <= 3;
        constexpr int NS = FS ? L + 1 : 2;
        double S[nsums<NS>()], ipf = 0.0;
        if constexpr (FS) {
#pragma unroll
            for (int t = 0; t < nsums<NS>(); ++t) S[t] = 0.0;
            ipf = far_scale(h.pf);
        }
        for (int k = k0; k < k1; k += PB) {
            PtInt<T> pt[PB];
            double qk[PB];
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                pt[b] = pts[k + b];
                qk[b] = q[k + b];
            }
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                if constexpr (FS) {
                    double x, y, z, sv[NS + 1];
                    eval_s<NS, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, ipf, pt[b].zeta2, pt[b].zeta,
                                  pt[b].lim, tab, qk[b], x, y, z, sv);
                    acc_S<NS>(sv, x, y, z, S);
                    continue;
                }
                if constexpr (L == 1) {  // q R_t with q R^(1), q R^(2) formed once
                    T x, y, z, Rn[3];
                    eval_Rn<2, T, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta,
                                  pt[b].lim, tab, x, y, z, Rn);
                    acc_V2<T>(qk[b], x, y, z, Rn, V);
                    continue;
                }
                if constexpr (L == 2) {  // q R_t with q R^(1..3) formed once
                    T x, y, z, Rn[4];
                    eval_Rn<3, T, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta,
                                  pt[b].lim, tab, x, y, z, Rn);
                    acc_V3<T>(qk[b], x, y, z, Rn, V);
                    continue;
                }
                if constexpr (L == 0) {  // q R_t with q R^(1) formed once
                    T x, y, z, Rn[2];
                    eval_Rn1<T, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta,
                                pt[b].lim, tab, x, y, z, Rn);
                    const double u = qk[b] * Rn[1];
                    V[0] = fma(qk[b], Rn[0], V[0]);
                    V[1] = fma(u, x, V[1]);
                    V[2] = fma(u, y, V[2]);
                    V[3] = fma(u, z, V[3]);
                    continue;
                }
                T R[NT];
                eval_R<L + 1, T, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta,
                                 pt[b].lim, tab, R);
#pragma unroll
                for (int t = 0; t < NT; ++t) V[t] = fma(qk[b], (double)R[t], V[t]);
            }
        }
        if constexpr (FS) fin_S<NS>(h.pf, S, V);
        if (ip < n_pairs) {
            double *o = d.vout + (size_t)ch * NT * n_pairs;
#pragma unroll
            for (int t = 0; t < NT; ++t) o[(size_t)t * n_pairs + ip] = V[t];
        }
    }
}

// per primitive pair: ga (3) and gb (3) from V' (sum of chunks)
template <int LA, int LB>
__global__ __launch_bounds__(64) void k_grad_contract(long long n, int nch, const double *__restrict__ vin, const int *__restrict__ ent_sp,
                                const int *__restrict__ ent_ij, const int *__restrict__ spa,
                                const int *__restrict__ spb, const int *__restrict__ snp, const int *__restrict__ soff,
                                const int *__restrict__ satom, const int *__restrict__ bfo,
                                const int *__restrict__ cnoff, const double *__restrict__ pexp,
                                const double *__restrict__ cn, const double *__restrict__ xyz,
                                const double *__restrict__ P, int nbf, double *__restrict__ gpair,
                                const unsigned long long *__restrict__ memb, const int *__restrict__ vperm) {
    constexpr int L = LA + LB, NT = ntuv(L + 1);
    // thread = slot of the pair order (V' is stored by slot), q = its list entry (null: the same)
    const long long qs = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (qs >= n) return;
    const long long q = vperm ? vperm[qs] : qs;
    if (memb && !((memb[ent_sp[q]] >> ent_ij[q]) & 1ull)) {  // entry of a merged list outside this term's list
        for (int d = 0; d < 6; ++d) gpair[(size_t)q * 6 + d] = 0.0;
        return;
    }
    // sums over the chunks in chunk order; the loads of one chunk are issued together
    double V[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) V[t] = 0.0;
    for (int c = 0; c < nch; ++c) {
        const double *__restrict__ vc = vin + (size_t)c * NT * n + qs;
        double u[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) u[t] = vc[(size_t)t * n];
#pragma unroll
        for (int t = 0; t < NT; ++t) V[t] += u[t];
    }
    int sp = ent_sp[q], ij = ent_ij[q];
    int a = spa[sp], b = spb[sp], i = ij >> 3, j = ij & 7;
    double ea = pexp[soff[a] + i], eb = pexp[soff[b] + j], p = ea + eb;
    const double *A = xyz + 3 * satom[a], *B = xyz + 3 * satom[b];
    double Pc[3] = {(ea * A[0] + eb * B[0]) / p, (ea * A[1] + eb * B[1]) / p, (ea * A[2] + eb * B[2]) / p};
    Herm1D<LA + 1, LB + 1> ex, ey, ez;
    double inv2p = 0.5 / p;
    ex.build(Pc[0] - A[0], Pc[0] - B[0], inv2p);
    ey.build(Pc[1] - A[1], Pc[1] - B[1], inv2p);
    ez.build(Pc[2] - A[2], Pc[2] - B[2], inv2p);
    double w = (a == b) ? -1.0 : -2.0;
    double g[6] = {0, 0, 0, 0, 0, 0};
    // sum over tuv of E^{a' b'}_{tuv} V_tuv for shifted Cartesian exponents; every loop here is
    // unrolled so that the exponents are constants and the tables stay in registers
    auto hv = [&](int ax, int ay, int az, int bx, int by, int bz) -> double {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t <= ax + bx; ++t)
#pragma unroll
            for (int u = 0; u <= ay + by; ++u) {
                double etu = ex.e[ax][bx][t] * ey.e[ay][by][u];
#pragma unroll
                for (int v = 0; v <= az + bz; ++v) s += etu * ez.e[az][bz][v] * V[tuv_idx(t, u, v)];
            }
        return s;
    };
#pragma unroll
    for (int mu = 0; mu < ncart(LA); ++mu) {
        int a3[3];
        cart_comp(LA, mu, a3[0], a3[1], a3[2]);
        double cmu = cn[cnoff[a] + mu * snp[a] + i];
#pragma unroll
        for (int nu = 0; nu < ncart(LB); ++nu) {
            int b3[3];
            cart_comp(LB, nu, b3[0], b3[1], b3[2]);
            double cf = w * P[(long long)(bfo[a] + mu) * nbf + bfo[b] + nu] * cmu * cn[cnoff[b] + nu * snp[b] + j];
            if (cf == 0.0) continue;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int ap[3] = {a3[0], a3[1], a3[2]};
                ap[d] += 1;
                double va = 2.0 * ea * hv(ap[0], ap[1], ap[2], b3[0], b3[1], b3[2]);
                if (a3[d] > 0) {
                    int am[3] = {a3[0], a3[1], a3[2]};
                    am[d] -= 1;
                    va -= a3[d] * hv(am[0], am[1], am[2], b3[0], b3[1], b3[2]);
                }
                int bp[3] = {b3[0], b3[1], b3[2]};
                bp[d] += 1;
                double vb = 2.0 * eb * hv(a3[0], a3[1], a3[2], bp[0], bp[1], bp[2]);
                if (b3[d] > 0) {
                    int bm[3] = {b3[0], b3[1], b3[2]};
                    bm[d] -= 1;
                    vb -= b3[d] * hv(a3[0], a3[1], a3[2], bm[0], bm[1], bm[2]);
                }
                g[d] += cf * va;
                g[3 + d] += cf * vb;
            }
        }
    }
    for (int d = 0; d < 6; ++d) gpair[(size_t)q * 6 + d] = g[d];
}

// The same per-pair (ga, gb) for classes with many Cartesian products (L >= 3): one wave per
// primitive pair.  V' and the three Hermite tables go to LDS, lane mu * ncart(LB) + nu takes
// one product of components, and the six sums over products are taken in that lane order,
// which is the loop order of k_grad_contract.
constexpr int GCW_WAVES = 4;
template <int LA, int LB>
__global__ __launch_bounds__(64 * GCW_WAVES) void k_grad_contract_w(
    long long n, int nch, const double *__restrict__ vin, const int *__restrict__ ent_sp,
    const int *__restrict__ ent_ij, const int *__restrict__ spa, const int *__restrict__ spb,
    const int *__restrict__ snp, const int *__restrict__ soff, const int *__restrict__ satom,
    const int *__restrict__ bfo, const int *__restrict__ cnoff, const double *__restrict__ pexp,
    const double *__restrict__ cn, const double *__restrict__ xyz, const double *__restrict__ P, int nbf,
    double *__restrict__ gpair, const unsigned long long *__restrict__ memb, const int *__restrict__ vperm) {
    constexpr int L = LA + LB, NT = ntuv(L + 1), IM = LA + 1, JM = LB + 1, TS = IM + JM + 1;
    constexpr int ES = herm1d_size<IM, JM>(), NA = ncart(LA), NB = ncart(LB);
    static_assert(NA * NB <= 64, "one lane per product of Cartesian components");
    __shared__ double sV[GCW_WAVES][NT];
    __shared__ double sE[GCW_WAVES][3][ES];
    __shared__ double sG[GCW_WAVES][6][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long qs = (long long)blockIdx.x * GCW_WAVES + w;  // slot of the pair order
    const long long q = qs < n && vperm ? vperm[qs] : qs;          // its list entry
    // an entry of a merged list outside this term's list contributes zeros
    const bool valid = qs < n && (!memb || ((memb[ent_sp[q]] >> ent_ij[q]) & 1ull));
    int a = 0, b = 0, i = 0, j = 0;
    double ea = 0.0, eb = 0.0;
    if (valid) {
        const int sp = ent_sp[q], ij = ent_ij[q];
        a = spa[sp];
        b = spb[sp];
        i = ij >> 3;
        j = ij & 7;
        ea = pexp[soff[a] + i];
        eb = pexp[soff[b] + j];
        if (lane < NT) sV[w][lane] = chunk_sum(vin + (size_t)lane * n + qs, (size_t)NT * n, nch);
        if (lane < 3) {
            const double p = ea + eb;
            const double Ad = xyz[3 * satom[a] + lane], Bd = xyz[3 * satom[b] + lane];
            const double Pd = (ea * Ad + eb * Bd) / p;
            herm1d_build_lds<IM, JM>(sE[w][lane], Pd - Ad, Pd - Bd, 0.5 / p);
        }
    }
    __syncthreads();
    double g[6] = {0, 0, 0, 0, 0, 0};
    if (valid && lane < NA * NB) {
        const int mu = lane / NB, nu = lane - mu * NB;
        int a3[3], b3[3];
        cart_comp(LA, mu, a3[0], a3[1], a3[2]);
        cart_comp(LB, nu, b3[0], b3[1], b3[2]);
        const double w2 = (a == b) ? -1.0 : -2.0;
        const double cf = w2 * P[(long long)(bfo[a] + mu) * nbf + bfo[b] + nu] * cn[cnoff[a] + mu * snp[a] + i] *
                          cn[cnoff[b] + nu * snp[b] + j];
        const double *ex = sE[w][0], *ey = sE[w][1], *ez = sE[w][2];
        const double *V = sV[w];
        auto hv = [&](int ax, int ay, int az, int bx, int by, int bz) -> double {
            double s = 0.0;
            for (int t = 0; t <= ax + bx; ++t)
                for (int u = 0; u <= ay + by; ++u) {
                    const double etu = ex[(ax * (JM + 1) + bx) * TS + t] * ey[(ay * (JM + 1) + by) * TS + u];
                    for (int v = 0; v <= az + bz; ++v)
                        s += etu * ez[(az * (JM + 1) + bz) * TS + v] * V[tuv_idx(t, u, v)];
                }
            return s;
        };
        if (cf != 0.0) {
            for (int d = 0; d < 3; ++d) {
                int ap[3] = {a3[0], a3[1], a3[2]};
                ap[d] += 1;
                double va = 2.0 * ea * hv(ap[0], ap[1], ap[2], b3[0], b3[1], b3[2]);
                if (a3[d] > 0) {
                    int am[3] = {a3[0], a3[1], a3[2]};
                    am[d] -= 1;
                    va -= a3[d] * hv(am[0], am[1], am[2], b3[0], b3[1], b3[2]);
                }
                int bp[3] = {b3[0], b3[1], b3[2]};
                bp[d] += 1;
                double vb = 2.0 * eb * hv(a3[0], a3[1], a3[2], bp[0], bp[1], bp[2]);
                if (b3[d] > 0) {
                    int bm[3] = {b3[0], b3[1], b3[2]};
                    bm[d] -= 1;
                    vb -= b3[d] * hv(a3[0], a3[1], a3[2], bm[0], bm[1], bm[2]);
                }
                g[d] = cf * va;
                g[3 + d] = cf * vb;
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) sG[w][d][lane] = g[d];
    __syncthreads();
    if (qs < n && lane < 6) {
        double acc = 0.0;
        for (int l = 0; l < NA * NB; ++l) acc += sG[w][lane][l];
        gpair[(size_t)q * 6 + lane] = acc;
    }
}

// per candidate shell pair: sum of its primitive pairs' (ga, gb) in list order
__global__ void k_grad_sp(long long sp0, long long nsp, long long cls_off, const int *__restrict__ spo,
                          const double *__restrict__ gpair, double *__restrict__ gsp, int add) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsp) return;
    long long sp = sp0 + s;
    int g0 = spo[sp], g1 = spo[sp + 1];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int g = g0; g < g1; ++g)
        for (int d = 0; d < 6; ++d) acc[d] += gpair[(size_t)(g - cls_off) * 6 + d];
    for (int d = 0; d < 6; ++d) gsp[(size_t)sp * 6 + d] = add ? gsp[(size_t)sp * 6 + d] + acc[d] : acc[d];
}

// -------------------------------------------------------------------------------------------
// 1/(2f) q^T dA_off q: per point k, (1/f) q_k sum_{l != k} q_l g'(r) (r_k - r_l)/r, partial rows
// g(r) = erf(z' r)/r, g'(r) = (2 z'/sqrt(pi)) exp(-z'^2 r^2)/r - erf(z' r)/r^2; for z' r >= 6.5
// the exponential term is below double precision relative to 1/r^2 and erf rounds to 1.
// -------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grad_aoff(const double *__restrict__ px, const double *__restrict__ py,
                                                   const double *__restrict__ pz, const double *__restrict__ zeta,
                                                   const double *__restrict__ q, int M, int chunk_len,
                                                   double *__restrict__ part) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = k < M ? k : M - 1;
    const double xk = px[kk], yk = py[kk], zk = pz[kk], zek = zeta[kk];
    const double hz = 0.5 * zek * zek;
    const int l0 = blockIdx.y * chunk_len;
    const int l1 = min(M, l0 + chunk_len);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int l = l0; l < l1; ++l) {
        double dx = xk - px[l], dy = yk - py[l], dz = zk - pz[l];
        double r2 = dx * dx + dy * dy + dz * dz;
        double zel = zeta[l];
        double g;  // g'(r)/r
        if (r2 * min(hz, 0.5 * zel * zel) >= 42.25) {
            double ri = rsqrt(r2);
            g = -ri * ri * ri;
        } else if (l == kk || r2 == 0.0) {
            g = 0.0;
        } else {
            double zp = zek * zel / sqrt(zek * zek + zel * zel);
            double r = sqrt(r2);
            double dg = 1.1283791670955125739 * zp * exp(-zp * zp * r2) / r - erf(zp * r) / r2;
            g = dg / r;
        }
        double w = q[l] * g;
        gx = fma(w, dx, gx);
        gy = fma(w, dy, gy);
        gz = fma(w, dz, gz);
    }
    if (k < M) {
        size_t base = (size_t)blockIdx.y * 3 * M;
        part[base + k] = gx;
        part[base + M + k] = gy;
        part[base + 2 * M + k] = gz;
    }
}

// -------------------------------------------------------------------------------------------
// final per-point gradient: A_off rows * q_k / f, c rows * (-q_k), plus the B term and the
// A_kk switching term (both sums over atoms)
// -------------------------------------------------------------------------------------------
__device__ __forceinline__ void point_atom_terms(double x, double y, double z, double zk, double qk, double Akk,
                                                 int I, int J, const double *__restrict__ xyz,
                                                 const double *__restrict__ Z, const double *__restrict__ rad,
                                                 double half_inv_f, double &gx, double &gy, double &gz) {
    double vx = x - xyz[3 * J], vy = y - xyz[3 * J + 1], vz = z - xyz[3 * J + 2];
    double d2 = vx * vx + vy * vy + vz * vz;
    if (d2 == 0.0) return;
    double d = sqrt(d2);
    // B: q_k Z_J d/dd [erf(zk d)/d] * v/d
    double dgb = (zk * d >= 6.5) ? -1.0 / d2
                                 : 1.1283791670955125739 * zk * exp(-zk * zk * d2) / d - erf(zk * d) / d2;
    double g = qk * Z[J] * dgb / d;
    // A_kk = c zk / prod S_wf: d A_kk = -A_kk sum dS_wf/S_wf
    if (J != I) {
        double RJ = rad[J];
        if (d < RJ + 6.0 / zk) {
            double am = RJ - d, ap = RJ + d;
            double sw = 0.5 * (erfc(zk * am) + erfc(zk * ap));
            double dsw = 0.56418958354775628695 * zk * (exp(-zk * zk * am * am) - exp(-zk * zk * ap * ap));
            g += half_inv_f * qk * qk * (-Akk) * dsw / sw / d;
        }
    }
    gx += g * vx;
    gy += g * vy;
    gz += g * vz;
}

__global__ __launch_bounds__(256) void k_grad_surf(int M, const double *__restrict__ px, const double *__restrict__ py,
                                                   const double *__restrict__ pz, const double *__restrict__ zeta,
                                                   const double *__restrict__ Akk, const int *__restrict__ keep,
                                                   int nsph, const double *__restrict__ q,
                                                   const double *__restrict__ xyz, const double *__restrict__ Z,
                                                   const double *__restrict__ rad, int N, double inv_f,
                                                   const double *__restrict__ part_a, int rows_a,
                                                   const double *__restrict__ part_c, int rows_c,
                                                   const double *__restrict__ dc, double *__restrict__ gs) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double qk = q[k];
    double g[3];
    for (int d = 0; d < 3; ++d) {
        double sa = 0.0, sc = 0.0;
        for (int r = 0; r < rows_a; ++r) sa += part_a[((size_t)r * 3 + d) * M + k];
        if (dc) {  // c term from dc_k = d c_k / d r_k given by the caller
            g[d] = fma(qk, dc[3 * k + d], inv_f * qk * sa);
            continue;
        }
        for (int r = 0; r < rows_c; ++r) sc += part_c[((size_t)r * 3 + d) * M + k];
        g[d] = inv_f * qk * sa - qk * sc;
    }
    double gx = 0.0, gy = 0.0, gz = 0.0;
    int I = keep[k] / nsph;
    for (int J = 0; J < N; ++J)
        point_atom_terms(px[k], py[k], pz[k], zeta[k], qk, Akk[k], I, J, xyz, Z, rad, 0.5 * inv_f, gx, gy, gz);
    gs[3 * k] = g[0] + gx;
    gs[3 * k + 1] = g[1] + gy;
    gs[3 * k + 2] = g[2] + gz;
}

// -------------------------------------------------------------------------------------------
// final per-atom gradient: -(point-atom terms) over all points + ga/gb over the atom's lists
// -------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grad_nuc(int N, int M, const double *__restrict__ px,
                                                  const double *__restrict__ py, const double *__restrict__ pz,
                                                  const double *__restrict__ zeta, const double *__restrict__ Akk,
                                                  const int *__restrict__ keep, int nsph, const double *__restrict__ q,
                                                  const double *__restrict__ xyz, const double *__restrict__ Z,
                                                  const double *__restrict__ rad, double inv_f,
                                                  const int *__restrict__ off_a, const int *__restrict__ lst_a,
                                                  const int *__restrict__ off_b, const int *__restrict__ lst_b,
                                                  const double *__restrict__ gsp, double *__restrict__ gn) {
    __shared__ double s[3][256];
    int J = blockIdx.x;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        double tx = 0.0, ty = 0.0, tz = 0.0;
        point_atom_terms(px[k], py[k], pz[k], zeta[k], q[k], Akk[k], keep[k] / nsph, J, xyz, Z, rad, 0.5 * inv_f, tx,
                         ty, tz);
        gx -= tx;
        gy -= ty;
        gz -= tz;
    }
    if (gsp) {
        for (int t = off_a[J] + threadIdx.x; t < off_a[J + 1]; t += blockDim.x) {
            const double *g = gsp + (size_t)lst_a[t] * 6;
            gx += g[0];
            gy += g[1];
            gz += g[2];
        }
        for (int t = off_b[J] + threadIdx.x; t < off_b[J + 1]; t += blockDim.x) {
            const double *g = gsp + (size_t)lst_b[t] * 6;
            gx += g[3];
            gy += g[4];
            gz += g[5];
        }
    }
    s[0][threadIdx.x] = gx;
    s[1][threadIdx.x] = gy;
    s[2][threadIdx.x] = gz;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int d = 0; d < 3; ++d) s[d][threadIdx.x] += s[d][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) gn[3 * J + d] = s[d][0];
}

// -------------------------------------------------------------------------------------------
// Work split into about 16,384 items (lane tiles x chunks of the other dimension): shorter
// chunks than the integral defaults balance the long gradient loops better (measured on the
// 600-atom protein: 145 ms per gradient at 4,096 items, 135 ms at 16,384).  A chunk is never
// shorter than `min_len`: classes with few pairs and small molecules would otherwise be cut into
// chunks of a few dozen points or pairs, whose partial sums cost more traffic than the work.
constexpr int GRAD_MIN_PTS = 512, GRAD_MIN_PAIRS = 512, GRAD_MIN_AOFF = 128;
static int chunk_for(long long n_work, long long n_lanes, int min_len) {
    int tiles = n_lanes > 0 ? div_up(n_lanes, 256) : 1;
    long long want = (16384 + tiles - 1) / tiles;
    if (want < 1) want = 1;
    long long len = (n_work + want - 1) / want;
    return (int)(len < min_len ? min_len : len);
}

// rows of the c-term point side for list `ls` (one per pair chunk per class)
static int grad_pts_chunk(long long n, int M) {
    return (chunk_for(n, M, GRAD_MIN_PAIRS) + REC_PAD - 1) / REC_PAD * REC_PAD;
}
static int grad_rows(pcm_mol *mol, ListSel ls) {
    const PairList &pl = mol->*ls;
    int rows = 0;
    for (int cl = 0; cl < NCLS; ++cl) {
        const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        rows += n ? div_up(n, grad_pts_chunk(n, mol->M)) : 0;
    }
    return rows;
}

// pair-side point chunk of class cl of list ls, and the V' / per-pair buffer sizes of the list
static int grad_v_chunk(pcm_mol *mol, ListSel ls, int cl) {
    const PairList &pl = mol->*ls;
    const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
    int c = chunk_for(mol->Mpad, n ? n : 1, GRAD_MIN_PTS);
    if (c < 32) c = 32;
    return (c + PT_BATCH - 1) / PT_BATCH * PT_BATCH;
}
static void grad_v_sizes(pcm_mol *mol, ListSel ls, size_t &vneed, size_t &gneed) {
    const PairList &pl = mol->*ls;
    for (int cl = 0; cl < NCLS; ++cl) {
        const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        const size_t v = (size_t)div_up(mol->Mpad, grad_v_chunk(mol, ls, cl)) * ntuv(CLS_LA[cl] + CLS_LB[cl] + 1) * n;
        vneed = std::max(vneed, v);
        gneed = std::max(gneed, (size_t)n * 6);
    }
}

// Per molecule of a gradient call: its inputs, outputs and the partial-row layout.
struct GradJob {
    pcm_mol *mol;
    const double *P, *q;
    double *g_nuc, *g_surf;
    int rows_a, rows_c, row0;  // A_off rows, c-term rows, next free c-term row
    double *part_a, *part_c;
    const double *dc = nullptr;  // given d c_k / d r_k: the c term's point side is not evaluated
};

// c term of one pair list for every molecule (charges already in qpad): per class, one launch of
// the point side (gc, partial rows of part_c from each job's row0 on) and one of the pair side
// (V' up to L+1) over all molecules, then per molecule the contraction to ga/gb and the sums per
// candidate shell pair into gsp (added when `add`).  The work split of a molecule does not
// depend on the other molecules, so a batched call gives the same bits as single calls.
// do_pts / do_pairs select the sides; with_c makes the point side also evaluate c (4-wide rows).
template <typename T, typename B>
static void grad_cterm(pcm_ctx *ctx, std::vector<GradJob> &jobs, ListSel ls, bool add, bool do_pts = true,
                       bool do_pairs = true, bool with_c = false) {
    const B *tab = sizeof(B) == 8 ? (const B *)ctx->boys64.p : (const B *)ctx->boys32.p;
    const std::string suffix = std::string("_") + prec_tag<T, B>();
    auto pts_of = [](pcm_mol *mol) -> const void * { return sizeof(T) == 8 ? (const void *)mol->pti64.p
                                                                             : (const void *)mol->pti32.p; };
    // V' chunking per molecule and class (vbuf and gpair were sized for every list in grad_run)
    const size_t nj = jobs.size();
    std::vector<std::array<int, NCLS>> chunk_v(nj);
    for (size_t i = 0; i < nj; ++i)
        for (int cl = 0; cl < NCLS; ++cl) chunk_v[i][cl] = grad_v_chunk(jobs[i].mol, ls, cl);
    for (int cl = 0; cl < NCLS; ++cl) {
        const int L = CLS_LA[cl] + CLS_LB[cl];
        const int stride = (int)rec_stride<T>(L);
        std::vector<GradPtsDesc> dp;
        std::vector<GradVDesc> dv;
        long long items_p = 0, items_v = 0;
        double work = 0.0;
        for (size_t i = 0; i < nj; ++i) {
            GradJob &j = jobs[i];
            pcm_mol *mol = j.mol;
            const PairList &pl = mol->*ls;
            const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
            if (!n) continue;
            const unsigned char *rec = pl.rec.p + pl.rec_off[cl];
            GradPtsDesc a{};
            a.rec = rec;
            a.pts = pts_of(mol);
            a.pperm = mol->pperm.p;
            a.part = j.part_c;
            a.base = items_p;
            a.stride = stride;
            a.n_pad = (int)((n + REC_PAD - 1) / REC_PAD * REC_PAD);
            a.chunk = grad_pts_chunk(n, mol->M);
            a.M = mol->M;
            a.ntile = div_up(mol->M, 256);
            a.row0 = j.row0;
            const int nch = div_up(n, a.chunk);
            items_p += (long long)a.ntile * nch;
            j.row0 += nch;
            dp.push_back(a);
            GradVDesc b{};
            b.rec = rec;
            b.perm = pair_order(pl, cl);
            b.pts = a.pts;
            b.q = mol->qpad.p;
            b.vout = mol->vbuf.p;
            b.base = items_v;
            b.stride = stride;
            b.n_pairs = (int)n;
            b.Mpad = mol->Mpad;
            b.chunk = chunk_v[i][cl];
            b.nptile = div_up(n, 256);
            items_v += (long long)b.nptile * div_up(mol->Mpad, b.chunk);
            dv.push_back(b);
            work += (double)n * mol->M;
        }
        if (!dp.empty()) {
            if (items_p > (1LL << 30) || items_v > (1LL << 30))
                throw PcmError{PCM_E_UNSUPPORTED, "gradient call too large for one launch per class"};
            const size_t pb = dp.size() * sizeof(GradPtsDesc), vb = dv.size() * sizeof(GradVDesc);
            std::vector<unsigned char> blob(pb + vb);
            std::memcpy(blob.data(), dp.data(), pb);
            std::memcpy(blob.data() + pb, dv.data(), vb);
            unsigned char *dev = (unsigned char *)upload_desc(ctx, blob.data(), blob.size());
            const GradPtsDesc *dpp = reinterpret_cast<const GradPtsDesc *>(dev);
            const GradVDesc *dvp = reinterpret_cast<const GradVDesc *>(dev + pb);
            const int nd = (int)dp.size();
            if (do_pts) {
                ProfScope ps(ctx, (with_c ? "esp_grad_pts_L" : "grad_pts_L") + std::to_string(L) + suffix, work);
                switch (L) {
#define GP_CASE(LL)                                                                                    \
    case LL:                                                                                           \
        if (with_c)                                                                                    \
            k_grad_pts<LL, T, B, true><<<int_grid(items_p), 256, 0, ctx->stream>>>(dpp, nd, items_p, tab); \
        else                                                                                           \
            k_grad_pts<LL, T, B, false><<<int_grid(items_p), 256, 0, ctx->stream>>>(dpp, nd, items_p, tab); \
        break;
                    GP_CASE(0) GP_CASE(1) GP_CASE(2) GP_CASE(3) GP_CASE(4)
#undef GP_CASE
                }
                HIP_LAUNCH_OK();
            }
            if (do_pairs) {
                ProfScope ps(ctx, "grad_v_L" + std::to_string(L) + suffix, work);
                switch (L) {
#define GV_CASE(LL)                                                                                    \
    case LL:                                                                                           \
        k_grad_v<LL, T, B><<<int_grid(items_v), 256, 0, ctx->stream>>>(dvp, nd, items_v, tab);         \
        break;
                    GV_CASE(0) GV_CASE(1) GV_CASE(2) GV_CASE(3) GV_CASE(4)
#undef GV_CASE
                }
                HIP_LAUNCH_OK();
            }
        }
        // per molecule: contraction of V' to (ga, gb) per primitive pair, sums per shell pair
        for (size_t i = 0; i < nj && do_pairs; ++i) {
            GradJob &j = jobs[i];
            pcm_mol *mol = j.mol;
            const PairList &pl = mol->*ls;
            const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
            const long long sp0 = mol->sp_cls_off[cl], ncs = mol->sp_cls_off[cl + 1] - sp0;
            if (!n) {
                if (ncs && !add)
                    HIP_OK(hipMemsetAsync(mol->gsp.p + sp0 * 6, 0, sizeof(double) * 6 * ncs, ctx->stream));
                continue;
            }
            const int nch = div_up(mol->Mpad, chunk_v[i][cl]);
            const int *es = pl.ent_sp.p + pl.cls_off[cl], *ei = pl.ent_ij.p + pl.cls_off[cl];
            const int *vp = pair_order(pl, cl);
            const int g = div_up(n, 64);
            const double *P = j.P;
            ProfScope ps2(ctx, "grad_contract", (double)n);
#define GC_CASE(CI, LA_, LB_)                                                                                      \
    case CI:                                                                                                       \
        k_grad_contract<LA_, LB_><<<g, 64, 0, ctx->stream>>>(n, nch, mol->vbuf.p, es, ei, mol->spa.p, mol->spb.p,  \
                                                             mol->snp.p, mol->soff.p, mol->satom.p, mol->bfo.p,    \
                                                             mol->cnoff.p, mol->pexp.p, mol->cn.p, mol->xyz.p,     \
                                                             P, mol->nbf, mol->gpair.p, nullptr, vp);                  \
        break;
#define GCW_CASE(CI, LA_, LB_)                                                                                     \
    case CI:                                                                                                       \
        k_grad_contract_w<LA_, LB_><<<div_up(n, GCW_WAVES), 64 * GCW_WAVES, 0, ctx->stream>>>(                      \
            n, nch, mol->vbuf.p, es, ei, mol->spa.p, mol->spb.p, mol->snp.p, mol->soff.p, mol->satom.p, mol->bfo.p, \
            mol->cnoff.p, mol->pexp.p, mol->cn.p, mol->xyz.p, P, mol->nbf, mol->gpair.p, nullptr, vp);              \
        break;
            switch (cl) {
                GC_CASE(0, 0, 0)
                GC_CASE(1, 0, 1)
                GC_CASE(2, 0, 2)
                GC_CASE(3, 1, 1)
                GCW_CASE(4, 1, 2)
                GCW_CASE(5, 2, 2)
            }
#undef GC_CASE
#undef GCW_CASE
            HIP_LAUNCH_OK();
            k_grad_sp<<<div_up(ncs, 128), 128, 0, ctx->stream>>>(sp0, ncs, pl.cls_off[cl], pl.spo.p, mol->gpair.p,
                                                                 mol->gsp.p, add ? 1 : 0);
            HIP_LAUNCH_OK();
        }
    }
}

static void grad_finish(pcm_ctx *ctx, std::vector<GradJob> &jobs, double inv_f);

// Eq. 14 at fixed density for one or more molecules: A off-diagonal rows, the c term of the
// list(s), then per point (g_surf) and per atom (g_nuc) with the B and switching terms
static void grad_run(pcm_ctx *ctx, std::vector<GradJob> &all, int prec) {
    const double inv_f = (ctx->prm.eps + ctx->prm.k_factor) / (ctx->prm.eps - 1.0);
    const bool dyn = prec == PCM_DYNAMIC;
    std::vector<GradJob> jobs;
    for (GradJob &j : all) {
        pcm_mol *mol = j.mol;
        const int M = mol->M;
        if (M == 0) {  // no surface charge: every term of Eq. 14 carries a factor q
            HIP_OK(hipMemsetAsync(j.g_nuc, 0, sizeof(double) * 3 * mol->N, ctx->stream));
            continue;
        }
        HIP_OK(hipMemcpyAsync(mol->qpad.p, j.q, sizeof(double) * M, hipMemcpyDeviceToDevice, ctx->stream));
        const int len_a = chunk_for(M, M, GRAD_MIN_AOFF);
        j.rows_a = div_up(M, len_a);
        j.rows_c = grad_rows(mol, &pcm_mol::esp) + (dyn ? grad_rows(mol, &pcm_mol::esp_w) : 0);
        j.row0 = 0;
        mol->part.ensure((size_t)(j.rows_a + j.rows_c + 1) * 3 * M);
        j.part_a = mol->part.p;
        j.part_c = mol->part.p + (size_t)j.rows_a * 3 * M;
        mol->gsp.ensure((size_t)mol->sp_cls_off[NCLS] * 6 + 6);
        size_t vneed = 0, gneed = 0;  // every list's needs, so that no buffer moves between launches
        grad_v_sizes(mol, &pcm_mol::esp, vneed, gneed);
        if (dyn) grad_v_sizes(mol, &pcm_mol::esp_w, vneed, gneed);
        mol->vbuf.ensure(vneed + 1);
        mol->gpair.ensure(gneed + 1);
        ProfScope psa(ctx, "grad_aoff", (double)M * M);
        k_grad_aoff<<<dim3(div_up(M, 256), j.rows_a), 256, 0, ctx->stream>>>(mol->px.p, mol->py.p, mol->pz.p,
                                                                               mol->zeta.p, j.q, M, len_a, j.part_a);
        HIP_LAUNCH_OK();
        jobs.push_back(j);
    }
    if (jobs.empty()) return;
    if (prec == PCM_MIXED) {
        grad_cterm<double, float>(ctx, jobs, &pcm_mol::esp, false);
    } else {
        grad_cterm<double, double>(ctx, jobs, &pcm_mol::esp, false);
        if (dyn) grad_cterm<float, float>(ctx, jobs, &pcm_mol::esp_w, true);
    }
    grad_finish(ctx, jobs, inv_f);
}

// per point (g_surf: A off-diagonal rows, c term, B and switching terms) and per atom (g_nuc)
static void grad_finish(pcm_ctx *ctx, std::vector<GradJob> &jobs, double inv_f) {
    for (GradJob &j : jobs) {
        pcm_mol *mol = j.mol;
        const int M = mol->M;
        const long long nsp = mol->sp_cls_off[NCLS];
        k_grad_surf<<<div_up(M, 256), 256, 0, ctx->stream>>>(M, mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p,
                                                             mol->Akk.p, mol->keep.p, mol->nsph, j.q, mol->xyz.p,
                                                             mol->Z.p, mol->rad.p, mol->N, inv_f, j.part_a, j.rows_a,
                                                             j.part_c, j.rows_c, j.dc, j.g_surf);
        HIP_LAUNCH_OK();
        k_grad_nuc<<<mol->N, 256, 0, ctx->stream>>>(mol->N, M, mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p,
                                                    mol->Akk.p, mol->keep.p, mol->nsph, j.q, mol->xyz.p, mol->Z.p,
                                                    mol->rad.p, inv_f, mol->atom_sp_off_a.p, mol->atom_sp_a.p,
                                                    mol->atom_sp_off_b.p, mol->atom_sp_b.p, nsp ? mol->gsp.p : nullptr,
                                                    j.g_nuc);
        HIP_LAUNCH_OK();
    }
}

void run_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, double *g_nuc, double *g_surf,
              int prec) {
    std::vector<GradJob> jobs{GradJob{mol, P, q, g_nuc, g_surf, 0, 0, 0, nullptr, nullptr}};
    grad_run(ctx, jobs, prec);
}

void run_grad_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &P,
                    const std::vector<const double *> &q, const std::vector<double *> &g_nuc,
                    const std::vector<double *> &g_surf, int prec) {
    std::vector<GradJob> jobs;
    for (size_t i = 0; i < mols.size(); ++i)
        jobs.push_back(GradJob{mols[i], P[i], q[i], g_nuc[i], g_surf[i], 0, 0, 0, nullptr, nullptr});
    grad_run(ctx, jobs, prec);
}

// -------------------------------------------------------------------------------------------
// One-pass forms.  c and dc_k = d c_k / d r_k come from the gradient's point side with the
// potential accumulated beside the derivative (the R^(n) it needs are a subset of those the
// derivative evaluates); the Fock sums V_tuv (t + u + v <= L) are the low orders of the V'_tuv
// the gradient's pair side accumulates, so one pass over the Eq. 18 list feeds both contractions;
// the Eq. 15 pairs outside that list need V up to L only, in a Fock pass of their own.
// -------------------------------------------------------------------------------------------
// c[k] = sum_r part[r][3][k], dc[3k + d] = -sum_r part[r][d][k] (rows in a fixed order)
__global__ __launch_bounds__(256) void k_field_sum(const double *__restrict__ part, int rows, int M,
                                                   double *__restrict__ c, double *__restrict__ dc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int r = 0; r < rows; ++r) {
        const double *p = part + (size_t)r * 4 * M + k;
        s0 += p[0];
        s1 += p[(size_t)M];
        s2 += p[2 * (size_t)M];
        s3 += p[3 * (size_t)M];
    }
    c[k] = s3;
    dc[3 * k] = -s0;
    dc[3 * k + 1] = -s1;
    dc[3 * k + 2] = -s2;
}

void run_esp_deriv(pcm_ctx *ctx, pcm_mol *mol, double *c, double *dc, int prec) {
    const int M = mol->M;
    const bool dyn = prec == PCM_DYNAMIC;
    GradJob j{mol, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, nullptr, nullptr};
    j.rows_c = grad_rows(mol, &pcm_mol::esp) + (dyn ? grad_rows(mol, &pcm_mol::esp_w) : 0);
    mol->part.ensure((size_t)(j.rows_c + 1) * 4 * M);
    j.part_c = mol->part.p;
    std::vector<GradJob> jobs{j};
    if (prec == PCM_MIXED) {
        grad_cterm<double, float>(ctx, jobs, &pcm_mol::esp, false, true, false, true);
    } else {
        grad_cterm<double, double>(ctx, jobs, &pcm_mol::esp, false, true, false, true);
        if (dyn) grad_cterm<float, float>(ctx, jobs, &pcm_mol::esp_w, false, true, false, true);
    }
    k_field_sum<<<grid_for(M, 256), 256, 0, ctx->stream>>>(mol->part.p, jobs[0].row0, M, c, dc);
    HIP_LAUNCH_OK();
}

// pair side over the Eq. 18 list, the Fock contraction (its Eq. 15 entries) and the gradient
// contraction of each class, sums per candidate shell pair into gsp
template <typename T, typename B>
static void fock_grad_pairs(pcm_ctx *ctx, pcm_mol *mol, const double *P, double *F, const PairList &pl, ListSel ls,
                            bool add) {
    const B *tab = sizeof(B) == 8 ? (const B *)ctx->boys64.p : (const B *)ctx->boys32.p;
    const std::string suffix = std::string("_") + prec_tag<T, B>();
    for (int cl = 0; cl < NCLS; ++cl) {
        const int L = CLS_LA[cl] + CLS_LB[cl];
        const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        const long long sp0 = mol->sp_cls_off[cl], ncs = mol->sp_cls_off[cl + 1] - sp0;
        if (!n) {
            if (ncs && !add) HIP_OK(hipMemsetAsync(mol->gsp.p + sp0 * 6, 0, sizeof(double) * 6 * ncs, ctx->stream));
            continue;
        }
        GradVDesc b{};
        b.rec = pl.rec.p + pl.rec_off[cl];
        b.perm = pair_order(pl, cl);
        b.pts = sizeof(T) == 8 ? (const void *)mol->pti64.p : (const void *)mol->pti32.p;
        b.q = mol->qpad.p;
        b.vout = mol->vbuf.p;
        b.base = 0;
        b.stride = (int)align16(sizeof(PairHdr<T>));
        b.n_pairs = (int)n;
        b.Mpad = mol->Mpad;
        b.chunk = grad_v_chunk(mol, ls, cl);
        b.nptile = div_up(n, 256);
        const int nch = div_up(mol->Mpad, b.chunk);
        const long long items = (long long)b.nptile * nch;
        if (items > (1LL << 30)) throw PcmError{PCM_E_UNSUPPORTED, "Fock + gradient pass too large for one launch"};
        const GradVDesc *dv = (const GradVDesc *)upload_desc(ctx, &b, sizeof(b));
        {
            ProfScope ps(ctx, "fock_grad_v_L" + std::to_string(L) + suffix, (double)n * mol->M);
            switch (L) {
#define GV_CASE(LL)                                                                                    \
    case LL:                                                                                           \
        k_grad_v<LL, T, B><<<int_grid(items), 256, 0, ctx->stream>>>(dv, 1, items, tab);               \
        break;
                GV_CASE(0) GV_CASE(1) GV_CASE(2) GV_CASE(3) GV_CASE(4)
#undef GV_CASE
            }
            HIP_LAUNCH_OK();
        }
        fock_contract_scatter(ctx, mol, pl, cl, mol->vbuf.p, nch, ntuv(L + 1), mol->m15.p, F);
        const int *es = pl.ent_sp.p + pl.cls_off[cl], *ei = pl.ent_ij.p + pl.cls_off[cl];
        const int *vp = pair_order(pl, cl);
        const unsigned long long *memb = mol->m18.p;
        ProfScope ps2(ctx, "grad_contract", (double)n);
#define GC_CASE(CI, LA_, LB_)                                                                                      \
    case CI:                                                                                                       \
        k_grad_contract<LA_, LB_><<<div_up(n, 64), 64, 0, ctx->stream>>>(                                          \
            n, nch, mol->vbuf.p, es, ei, mol->spa.p, mol->spb.p, mol->snp.p, mol->soff.p, mol->satom.p, mol->bfo.p, \
            mol->cnoff.p, mol->pexp.p, mol->cn.p, mol->xyz.p, P, mol->nbf, mol->gpair.p, memb, vp);                 \
        break;
#define GCW_CASE(CI, LA_, LB_)                                                                                     \
    case CI:                                                                                                       \
        k_grad_contract_w<LA_, LB_><<<div_up(n, GCW_WAVES), 64 * GCW_WAVES, 0, ctx->stream>>>(                      \
            n, nch, mol->vbuf.p, es, ei, mol->spa.p, mol->spb.p, mol->snp.p, mol->soff.p, mol->satom.p, mol->bfo.p, \
            mol->cnoff.p, mol->pexp.p, mol->cn.p, mol->xyz.p, P, mol->nbf, mol->gpair.p, memb, vp);                 \
        break;
        switch (cl) {
            GC_CASE(0, 0, 0)
            GC_CASE(1, 0, 1)
            GC_CASE(2, 0, 2)
            GC_CASE(3, 1, 1)
            GCW_CASE(4, 1, 2)
            GCW_CASE(5, 2, 2)
        }
#undef GC_CASE
#undef GCW_CASE
        HIP_LAUNCH_OK();
        k_grad_sp<<<div_up(ncs, 128), 128, 0, ctx->stream>>>(sp0, ncs, pl.cls_off[cl], pl.spo.p, mol->gpair.p,
                                                             mol->gsp.p, add ? 1 : 0);
        HIP_LAUNCH_OK();
    }
}

void run_fock_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, const double *dc, double *F,
                   double *g_nuc, double *g_surf, int prec) {
    const double inv_f = (ctx->prm.eps + ctx->prm.k_factor) / (ctx->prm.eps - 1.0);
    const int M = mol->M;
    const bool dyn = prec == PCM_DYNAMIC;
    HIP_OK(hipMemcpyAsync(mol->qpad.p, q, sizeof(double) * M, hipMemcpyDeviceToDevice, ctx->stream));
    const int len_a = chunk_for(M, M, GRAD_MIN_AOFF);
    const int rows_a = div_up(M, len_a);
    mol->part.ensure((size_t)(rows_a + 1) * 3 * M);
    mol->gsp.ensure((size_t)mol->sp_cls_off[NCLS] * 6 + 6);
    // V', per-pair blocks and gradient rows sized for every part before the first launch
    size_t vneed = 0, gneed = 0, fneed = 0;
    for (ListSel ls : {&pcm_mol::fg, &pcm_mol::fg_w}) {
        const PairList &pl = mol->*ls;
        grad_v_sizes(mol, ls, vneed, gneed);
        for (int cl = 0; cl < NCLS; ++cl)
            fneed = std::max(fneed, (size_t)(pl.cls_off[cl + 1] - pl.cls_off[cl]) * ncart(CLS_LA[cl]) *
                                        ncart(CLS_LB[cl]));
    }
    mol->vbuf.ensure(vneed + 1);
    mol->gpair.ensure(gneed + 1);
    mol->fprim.ensure(fneed + 1);
    fock_buffers(mol, &pcm_mol::fo);
    fock_buffers(mol, &pcm_mol::fo_w);
    {
        ProfScope psa(ctx, "grad_aoff", (double)M * M);
        k_grad_aoff<<<dim3(div_up(M, 256), rows_a), 256, 0, ctx->stream>>>(mol->px.p, mol->py.p, mol->pz.p,
                                                                            mol->zeta.p, q, M, len_a, mol->part.p);
        HIP_LAUNCH_OK();
    }
    if (prec == PCM_MIXED) {
        fock_grad_pairs<double, float>(ctx, mol, P, F, mol->fg, &pcm_mol::fg, false);
    } else {
        fock_grad_pairs<double, double>(ctx, mol, P, F, mol->fg, &pcm_mol::fg, false);
        if (dyn) fock_grad_pairs<float, float>(ctx, mol, P, F, mol->fg_w, &pcm_mol::fg_w, true);
    }
    // the Eq. 15 pairs outside the Eq. 18 list contribute to F only
    run_fock_lists(ctx, mol, q, F, prec, &pcm_mol::fo, &pcm_mol::fo_w);
    GradJob j{mol, P, q, g_nuc, g_surf, rows_a, 0, 0, mol->part.p, nullptr};
    j.dc = dc;
    std::vector<GradJob> all{j};
    grad_finish(ctx, all, inv_f);
}
