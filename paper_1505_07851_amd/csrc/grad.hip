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

// -------------------------------------------------------------------------------------------
// gc: g_surf contribution of the c term, partial over a chunk of pairs (3 rows per chunk)
// -------------------------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(256) void k_grad_pts(const unsigned char *__restrict__ rec, int stride, int n_pad,
                                                  int chunk_len, const PtInt<T> *__restrict__ pts, int M,
                                                  const T *__restrict__ boys_g, double *__restrict__ part, int row0) {
    constexpr int NT = ntuv(L), PB = pair_batch<L + 1>();
    __shared__ T tab[boys_lds_size<T, L + 1>()];
    load_boys<T, L + 1>(tab, boys_g);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const PtInt<T> me = pts[k < M ? k : M - 1];
    const int p0 = blockIdx.y * chunk_len;
    const int p1 = min(n_pad, p0 + chunk_len);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int ip = p0; ip < p1; ip += PB) {
        PairHdr<T> h[PB];
        T D[PB][NT];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const unsigned char *r = rec + (size_t)(ip + b) * stride;
            h[b] = *reinterpret_cast<const PairHdr<T> *>(r);
            const T *d = reinterpret_cast<const T *>(r + sizeof(PairHdr<T>));
#pragma unroll
            for (int t = 0; t < NT; ++t) D[b][t] = d[t];
        }
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            T R[ntuv(L + 1)];
            eval_R<L + 1, T>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim, tab, R);
            if constexpr (sizeof(T) == 8) {  // FP64: straight into the accumulators
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    gx = fma(D[b][t], R[TuvShift<L>::x(t)], gx);
                    gy = fma(D[b][t], R[TuvShift<L>::y(t)], gy);
                    gz = fma(D[b][t], R[TuvShift<L>::z(t)], gz);
                }
            } else {  // FP32 evaluation, one FP64 add per pair
                T sx = T(0), sy = T(0), sz = T(0);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    sx = fma(D[b][t], R[TuvShift<L>::x(t)], sx);
                    sy = fma(D[b][t], R[TuvShift<L>::y(t)], sy);
                    sz = fma(D[b][t], R[TuvShift<L>::z(t)], sz);
                }
                gx += (double)sx;
                gy += (double)sy;
                gz += (double)sz;
            }
        }
    }
    if (k < M) {
        size_t base = (size_t)(row0 + blockIdx.y) * 3 * M;
        part[base + k] = gx;
        part[base + M + k] = gy;
        part[base + 2 * M + k] = gz;
    }
}

// -------------------------------------------------------------------------------------------
// V'_tuv up to L+1 per pair (lane = pair), weights q_k; same as the Fock accumulation
// -------------------------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(256) void k_grad_v(const unsigned char *__restrict__ rec, int stride, int n_pairs,
                                                const PtInt<T> *__restrict__ pts, const double *__restrict__ q,
                                                int Mpad, int chunk_len, const T *__restrict__ boys_g,
                                                double *__restrict__ vout) {
    __shared__ T tab[boys_lds_size<T, L + 1>()];
    load_boys<T, L + 1>(tab, boys_g);
    constexpr int NT = ntuv(L + 1);
    const int ip = blockIdx.x * blockDim.x + threadIdx.x;
    const int ipp = ip < n_pairs ? ip : n_pairs - 1;
    const PairHdr<T> h = *reinterpret_cast<const PairHdr<T> *>(rec + (size_t)ipp * stride);
    const int k0 = blockIdx.y * chunk_len;
    const int k1 = min(Mpad, k0 + chunk_len);
    double V[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) V[t] = 0.0;
    // points per batch: fewer for the larger V' sets so that more waves stay resident
    constexpr int PB = L <= 1 ? PT_BATCH : (L == 2 ? 2 : 1);
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
            T R[NT];
            eval_R<L + 1, T>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta, pt[b].lim,
                             tab, R);
#pragma unroll
            for (int t = 0; t < NT; ++t) V[t] = fma(qk[b], (double)R[t], V[t]);
        }
    }
    if (ip < n_pairs) {
        double *o = vout + (size_t)blockIdx.y * NT * n_pairs;
#pragma unroll
        for (int t = 0; t < NT; ++t) o[(size_t)t * n_pairs + ip] = V[t];
    }
}

// per primitive pair: ga (3) and gb (3) from V' (sum of chunks)
template <int LA, int LB>
__global__ void k_grad_contract(long long n, int nch, const double *__restrict__ vin, const int *__restrict__ ent_sp,
                                const int *__restrict__ ent_ij, const int *__restrict__ spa,
                                const int *__restrict__ spb, const int *__restrict__ snp, const int *__restrict__ soff,
                                const int *__restrict__ satom, const int *__restrict__ bfo,
                                const int *__restrict__ cnoff, const double *__restrict__ pexp,
                                const double *__restrict__ cn, const double *__restrict__ xyz,
                                const double *__restrict__ P, int nbf, double *__restrict__ gpair) {
    constexpr int L = LA + LB, NT = ntuv(L + 1);
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double V[NT];
    for (int t = 0; t < NT; ++t) {
        double s = 0.0;
        for (int c = 0; c < nch; ++c) s += vin[((size_t)c * NT + t) * n + q];
        V[t] = s;
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
    // sum over tuv of E^{a' b'}_{tuv} V_tuv for shifted Cartesian exponents
    auto hv = [&](int ax, int ay, int az, int bx, int by, int bz) -> double {
        double s = 0.0;
        for (int t = 0; t <= ax + bx; ++t)
            for (int u = 0; u <= ay + by; ++u) {
                double etu = ex.e[ax][bx][t] * ey.e[ay][by][u];
                for (int v = 0; v <= az + bz; ++v) s += etu * ez.e[az][bz][v] * V[tuv_idx(t, u, v)];
            }
        return s;
    };
    for (int mu = 0; mu < ncart(LA); ++mu) {
        int a3[3];
        cart_comp(LA, mu, a3[0], a3[1], a3[2]);
        double cmu = cn[cnoff[a] + mu * snp[a] + i];
        for (int nu = 0; nu < ncart(LB); ++nu) {
            int b3[3];
            cart_comp(LB, nu, b3[0], b3[1], b3[2]);
            double cf = w * P[(long long)(bfo[a] + mu) * nbf + bfo[b] + nu] * cmu * cn[cnoff[b] + nu * snp[b] + j];
            if (cf == 0.0) continue;
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
    double *__restrict__ gpair) {
    constexpr int L = LA + LB, NT = ntuv(L + 1), IM = LA + 1, JM = LB + 1, TS = IM + JM + 1;
    constexpr int ES = herm1d_size<IM, JM>(), NA = ncart(LA), NB = ncart(LB);
    static_assert(NA * NB <= 64, "one lane per product of Cartesian components");
    __shared__ double sV[GCW_WAVES][NT];
    __shared__ double sE[GCW_WAVES][3][ES];
    __shared__ double sG[GCW_WAVES][6][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long q = (long long)blockIdx.x * GCW_WAVES + w;
    const bool valid = q < n;
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
        if (lane < NT) {
            double acc = 0.0;
            for (int c = 0; c < nch; ++c) acc += vin[((size_t)c * NT + lane) * n + q];
            sV[w][lane] = acc;
        }
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
    if (valid && lane < 6) {
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
                                                   double *__restrict__ gs) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double qk = q[k];
    double g[3];
    for (int d = 0; d < 3; ++d) {
        double sa = 0.0, sc = 0.0;
        for (int r = 0; r < rows_a; ++r) sa += part_a[((size_t)r * 3 + d) * M + k];
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
// work split into about 16,384 items (lane tiles x chunks of the other dimension): shorter
// chunks than the integral defaults balance the long gradient loops better (measured on the
// 600-atom protein: 145 ms per gradient at 4,096 items, 135 ms at 16,384)
static int chunk_for(long long n_work, long long n_lanes) {
    int tiles = n_lanes > 0 ? div_up(n_lanes, 256) : 1;
    long long want = (16384 + tiles - 1) / tiles;
    if (want < 1) want = 1;
    long long len = (n_work + want - 1) / want;
    return (int)(len < 16 ? 16 : len);
}

// rows of the c-term point side for list `ls` (one per pair chunk per class)
static int grad_pts_chunk(long long n, int M) { return (chunk_for(n, M) + REC_PAD - 1) / REC_PAD * REC_PAD; }
static int grad_rows(pcm_mol *mol, ListSel ls) {
    const PairList &pl = mol->*ls;
    int rows = 0;
    for (int cl = 0; cl < NCLS; ++cl) {
        const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        rows += n ? div_up(n, grad_pts_chunk(n, mol->M)) : 0;
    }
    return rows;
}

// c term of one pair list (charges already in qpad): the point side (gc) as partial rows of part_c
// from row0 on, the pair side (ga, gb) summed per candidate shell pair into gsp (added when `add`)
template <typename T>
static void grad_cterm(pcm_ctx *ctx, pcm_mol *mol, const double *P, ListSel ls, double *part_c, int &row0,
                       bool add) {
    PairList &pl = mol->*ls;
    const int M = mol->M, Mpad = mol->Mpad;
    const T *tab = sizeof(T) == 8 ? (const T *)ctx->boys64.p : (const T *)ctx->boys32.p;
    const PtInt<T> *pts = reinterpret_cast<const PtInt<T> *>(sizeof(T) == 8 ? mol->pti64.p : mol->pti32.p);
    const char *suffix = sizeof(T) == 8 ? "_f64" : "_f32";
    for (int cl = 0; cl < NCLS; ++cl) {
        const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        if (!n) continue;
        const int L = CLS_LA[cl] + CLS_LB[cl];
        const int chunk = grad_pts_chunk(n, M);
        const int nch = div_up(n, chunk);
        const int n_pad = (int)((n + REC_PAD - 1) / REC_PAD * REC_PAD);
        dim3 grid(div_up(M, 256), nch);
        const unsigned char *rec = pl.rec.p + pl.rec_off[cl];
        const int stride = (int)rec_stride<T>(L);
        ProfScope ps(ctx, "grad_pts_L" + std::to_string(L) + suffix, (double)n * M);
        switch (L) {
#define GP_CASE(LL)                                                                                                 \
    case LL:                                                                                                        \
        k_grad_pts<LL, T><<<grid, 256, 0, ctx->stream>>>(rec, stride, n_pad, chunk, pts, M, tab, part_c, row0);     \
        break;
            GP_CASE(0) GP_CASE(1) GP_CASE(2) GP_CASE(3) GP_CASE(4)
#undef GP_CASE
        }
        HIP_LAUNCH_OK();
        row0 += nch;
    }
    // pair side: V' (L+1) per pair, contraction, per shell pair
    size_t vneed = 0, gneed = 0;
    int chunk_v[NCLS];
    for (int cl = 0; cl < NCLS; ++cl) {
        const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        chunk_v[cl] = chunk_for(Mpad, n ? n : 1);
        if (chunk_v[cl] < 32) chunk_v[cl] = 32;
        chunk_v[cl] = (chunk_v[cl] + PT_BATCH - 1) / PT_BATCH * PT_BATCH;
        const size_t v = (size_t)div_up(Mpad, chunk_v[cl]) * ntuv(CLS_LA[cl] + CLS_LB[cl] + 1) * n;
        vneed = v > vneed ? v : vneed;
        gneed = (size_t)n * 6 > gneed ? (size_t)n * 6 : gneed;
    }
    mol->vbuf.ensure(vneed + 1);
    mol->gpair.ensure(gneed + 1);
    for (int cl = 0; cl < NCLS; ++cl) {
        const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        const long long sp0 = mol->sp_cls_off[cl], ncs = mol->sp_cls_off[cl + 1] - sp0;
        if (!n) {
            if (ncs && !add) HIP_OK(hipMemsetAsync(mol->gsp.p + sp0 * 6, 0, sizeof(double) * 6 * ncs, ctx->stream));
            continue;
        }
        const int L = CLS_LA[cl] + CLS_LB[cl];
        const int nch = div_up(Mpad, chunk_v[cl]);
        const unsigned char *rec = pl.rec.p + pl.rec_off[cl];
        const int stride = (int)rec_stride<T>(L);
        {
            ProfScope ps(ctx, "grad_v_L" + std::to_string(L) + suffix, (double)n * M);
            dim3 grid(div_up(n, 256), nch);
            switch (L) {
#define GV_CASE(LL)                                                                                                \
    case LL:                                                                                                       \
        k_grad_v<LL, T><<<grid, 256, 0, ctx->stream>>>(rec, stride, (int)n, pts, mol->qpad.p, Mpad, chunk_v[cl],   \
                                                       tab, mol->vbuf.p);                                           \
        break;
                GV_CASE(0) GV_CASE(1) GV_CASE(2) GV_CASE(3) GV_CASE(4)
#undef GV_CASE
            }
            HIP_LAUNCH_OK();
        }
        const int *es = pl.ent_sp.p + pl.cls_off[cl], *ei = pl.ent_ij.p + pl.cls_off[cl];
        const int g = div_up(n, 64);
        ProfScope ps2(ctx, "grad_contract", (double)n);
#define GC_CASE(CI, LA_, LB_)                                                                                      \
    case CI:                                                                                                       \
        k_grad_contract<LA_, LB_><<<g, 64, 0, ctx->stream>>>(n, nch, mol->vbuf.p, es, ei, mol->spa.p, mol->spb.p,  \
                                                             mol->snp.p, mol->soff.p, mol->satom.p, mol->bfo.p,    \
                                                             mol->cnoff.p, mol->pexp.p, mol->cn.p, mol->xyz.p,     \
                                                             P, mol->nbf, mol->gpair.p);                               \
        break;
#define GCW_CASE(CI, LA_, LB_)                                                                                     \
    case CI:                                                                                                       \
        k_grad_contract_w<LA_, LB_><<<div_up(n, GCW_WAVES), 64 * GCW_WAVES, 0, ctx->stream>>>(                      \
            n, nch, mol->vbuf.p, es, ei, mol->spa.p, mol->spb.p, mol->snp.p, mol->soff.p, mol->satom.p, mol->bfo.p, \
            mol->cnoff.p, mol->pexp.p, mol->cn.p, mol->xyz.p, P, mol->nbf, mol->gpair.p);                           \
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

// Eq. 14 at fixed density: A off-diagonal rows, the c term of the list(s), then per point
// (g_surf) and per atom (g_nuc) with the B and switching terms
static void grad_launch(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, double *g_nuc, double *g_surf,
                        int prec) {
    const int M = mol->M;
    const double inv_f = (ctx->prm.eps + ctx->prm.k_factor) / (ctx->prm.eps - 1.0);
    if (M == 0) {  // no surface charge: every term of Eq. 14 carries a factor q
        HIP_OK(hipMemsetAsync(g_nuc, 0, sizeof(double) * 3 * mol->N, ctx->stream));
        return;
    }
    const bool dyn = prec == PCM_DYNAMIC;
    HIP_OK(hipMemcpyAsync(mol->qpad.p, q, sizeof(double) * M, hipMemcpyDeviceToDevice, ctx->stream));
    const int len_a = chunk_for(M, M);
    const int rows_a = div_up(M, len_a);
    const int rows_c = grad_rows(mol, &pcm_mol::esp) + (dyn ? grad_rows(mol, &pcm_mol::esp_w) : 0);
    mol->part.ensure((size_t)(rows_a + rows_c + 1) * 3 * M);
    double *part_a = mol->part.p, *part_c = mol->part.p + (size_t)rows_a * 3 * M;
    const long long nsp = mol->sp_cls_off[NCLS];
    mol->gsp.ensure((size_t)nsp * 6 + 6);
    {
        ProfScope psa(ctx, "grad_aoff", (double)M * M);
        k_grad_aoff<<<dim3(div_up(M, 256), rows_a), 256, 0, ctx->stream>>>(mol->px.p, mol->py.p, mol->pz.p,
                                                                             mol->zeta.p, q, M, len_a, part_a);
        HIP_LAUNCH_OK();
    }
    int row0 = 0;
    if (prec == PCM_MIXED) {
        grad_cterm<float>(ctx, mol, P, &pcm_mol::esp, part_c, row0, false);
    } else {
        grad_cterm<double>(ctx, mol, P, &pcm_mol::esp, part_c, row0, false);
        if (dyn) grad_cterm<float>(ctx, mol, P, &pcm_mol::esp_w, part_c, row0, true);
    }
    k_grad_surf<<<div_up(M, 256), 256, 0, ctx->stream>>>(M, mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p, mol->Akk.p,
                                                         mol->keep.p, mol->nsph, q, mol->xyz.p, mol->Z.p, mol->rad.p,
                                                         mol->N, inv_f, part_a, rows_a, part_c, rows_c, g_surf);
    HIP_LAUNCH_OK();
    k_grad_nuc<<<mol->N, 256, 0, ctx->stream>>>(mol->N, M, mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p, mol->Akk.p,
                                                mol->keep.p, mol->nsph, q, mol->xyz.p, mol->Z.p, mol->rad.p, inv_f,
                                                mol->atom_sp_off_a.p, mol->atom_sp_a.p, mol->atom_sp_off_b.p,
                                                mol->atom_sp_b.p, nsp ? mol->gsp.p : nullptr, g_nuc);
    HIP_LAUNCH_OK();
}

void run_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, double *g_nuc, double *g_surf,
              int prec) {
    grad_launch(ctx, mol, P, q, g_nuc, g_surf, prec);
}
