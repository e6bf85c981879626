/*
 * pcm_oracle.c -- plain, slow, FP64 CPU reference for the C-PCM / ISWIG
 * solvation path of Liu, Luehr, Kulik and Martinez, "Quantum Chemistry for
 * Solvated Molecules on GPUs using Polarizable Continuum Models"
 * (arXiv:1505.07851).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP library: integrals here follow the Obara-Saika vertical recursion
 * plus the horizontal (centre-transfer) relation, while the GPU path uses a
 * Hermite (McMurchie-Davidson) expansion.
 *
 * Every function below cites the passage of the paper it follows:
 *   Sec. 2, Eq. 1      response equation A q = -f (B z + c)
 *   Sec. 2, Eq. 2, 8   off-diagonal A with the combined exponent
 *   Sec. 2, Eq. 3      diagonal of A (constant read as sqrt(2/pi), passed in)
 *   Sec. 2, Eq. 4      nucleus - surface interaction B
 *   Sec. 2, Eqs. 5, 6  c = sum P L, L = -(mu|J_k|nu)
 *   Sec. 2, Eq. 7      Gaussian exponent of a surface point
 *   Sec. 2, Eq. 9      ISWIG switching function
 *   Sec. 2, Eq. 10     Fock correction sum_k q_k L^k
 *   Sec. 2, Eqs. 11-12 contracted from primitive integrals
 *   Sec. 2, Eq. 14     gradient at fixed density
 *   Sec. 4a, Eqs. 15, 18  Schwarz-like primitive-pair screening
 *   Sec. 4b-ii         randomized block-Jacobi partition
 * Units: bohr, hartree, elementary charge.  Build: gcc -O2 -fopenmp
 * -ffp-contract=off (no fused multiply-add, so the partition's ranking
 * values are plain IEEE double expressions).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LT_MAX 6 /* highest total angular momentum in a recursion table */

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian component `idx` of shell l in lexicographic order
 * (x, y, z; xx, xy, xz, yy, yz, zz). */
static void cart(int l, int idx, int *ax, int *ay, int *az) {
    int n = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (n == idx) { *ax = x; *ay = y; *az = l - x - y; return; }
            ++n;
        }
    *ax = *ay = *az = -1;
}

static double dfact_odd(int n) { /* (2n-1)!! with (-1)!! = 1 */
    double r = 1.0;
    for (int k = 2 * n - 1; k > 1; k -= 2) r *= (double)k;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt, m = 0..mmax.        */
/* Series for the top order, then downward recursion (T <= 30); erf form of  */
/* F_0 and upward recursion above.                                           */
/* ------------------------------------------------------------------------ */
void or_boys(int mmax, double T, double *F) {
    if (T <= 30.0) {
        double term = 1.0 / (2 * mmax + 1), sum = term;
        for (int i = 1; i < 2000; ++i) {
            term *= 2.0 * T / (double)(2 * mmax + 2 * i + 1);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        double e = exp(-T);
        F[mmax] = e * sum;
        for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) / (2 * m + 1);
    } else {
        double e = exp(-T);
        F[0] = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) / (2.0 * T);
    }
}

/* ------------------------------------------------------------------------ */
/* Primitive integrals [a | erf(zeta|r-C|)/|r-C| | b]  (Sec. 2, Eq. 6 for    */
/* one primitive pair, Eq. 12).  Obara-Saika: the attenuated operator keeps  */
/* the nuclear-attraction recursion with auxiliary integrals                 */
/*   Theta^(m) = (2 pi / p) K u^(m+1/2) F_m(p u |P-C|^2),  u = z^2/(z^2+p),   */
/* which follows from erf(z r)/r = 2/sqrt(pi) int_0^z exp(-s^2 r^2) ds.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double v[LT_MAX + 1][LT_MAX + 1][LT_MAX + 1][LT_MAX + 1]; /* [m][ax][ay][az] */
    double AB[3];
} os_table;

static void os_build(int Lt, const double *A, double ea, const double *B, double eb,
                     const double *C, double zeta, os_table *T) {
    double p = ea + eb;
    double P[3], PA[3], PC[3], ab2 = 0.0, pc2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        P[d] = (ea * A[d] + eb * B[d]) / p;
        PA[d] = P[d] - A[d];
        PC[d] = P[d] - C[d];
        T->AB[d] = A[d] - B[d];
        ab2 += (A[d] - B[d]) * (A[d] - B[d]);
        pc2 += PC[d] * PC[d];
    }
    double K = exp(-ea * eb / p * ab2);
    double u = zeta * zeta / (zeta * zeta + p);
    double F[LT_MAX + 2];
    or_boys(Lt, p * u * pc2, F);
    double pre = 2.0 * M_PI / p * K * sqrt(u), um = 1.0;
    for (int m = 0; m <= Lt; ++m) { T->v[m][0][0][0] = pre * um * F[m]; um *= u; }
    double inv2p = 0.5 / p;
    for (int N = 1; N <= Lt; ++N)
        for (int ax = N; ax >= 0; --ax)
            for (int ay = N - ax; ay >= 0; --ay) {
                int az = N - ax - ay, a[3] = {ax, ay, az};
                int i = ax > 0 ? 0 : (ay > 0 ? 1 : 2);
                int a1[3] = {ax, ay, az};
                a1[i] -= 1; /* a - 1_i */
                for (int m = 0; m <= Lt - N; ++m) {
                    double val = PA[i] * T->v[m][a1[0]][a1[1]][a1[2]] - PC[i] * T->v[m + 1][a1[0]][a1[1]][a1[2]];
                    if (a1[i] > 0) {
                        int a2[3] = {a1[0], a1[1], a1[2]};
                        a2[i] -= 1;
                        val += a1[i] * inv2p * (T->v[m][a2[0]][a2[1]][a2[2]] - T->v[m + 1][a2[0]][a2[1]][a2[2]]);
                    }
                    T->v[m][a[0]][a[1]][a[2]] = val;
                }
            }
}

/* centre transfer: [a|b] = [a+1_i|b-1_i] + (A-B)_i [a|b-1_i] */
static double os_hrr(const os_table *T, int ax, int ay, int az, int bx, int by, int bz) {
    if (ax < 0 || ay < 0 || az < 0 || bx < 0 || by < 0 || bz < 0) return 0.0;
    if (bx > 0) return os_hrr(T, ax + 1, ay, az, bx - 1, by, bz) + T->AB[0] * os_hrr(T, ax, ay, az, bx - 1, by, bz);
    if (by > 0) return os_hrr(T, ax, ay + 1, az, bx, by - 1, bz) + T->AB[1] * os_hrr(T, ax, ay, az, bx, by - 1, bz);
    if (bz > 0) return os_hrr(T, ax, ay, az + 1, bx, by, bz - 1) + T->AB[2] * os_hrr(T, ax, ay, az, bx, by, bz - 1);
    return T->v[0][ax][ay][az];
}

/* out[ia*ncart(lb)+ib] = [chi_a^ia | J_C | chi_b^ib], unnormalised primitives */
void or_prim_block(int la, int lb, const double *A, double ea, const double *B, double eb,
                   const double *C, double zeta, double *out) {
    os_table T;
    os_build(la + lb, A, ea, B, eb, C, zeta, &T);
    int na = ncart(la), nb = ncart(lb);
    for (int i = 0; i < na; ++i) {
        int ax, ay, az;
        cart(la, i, &ax, &ay, &az);
        for (int j = 0; j < nb; ++j) {
            int bx, by, bz;
            cart(lb, j, &bx, &by, &bz);
            out[i * nb + j] = os_hrr(&T, ax, ay, az, bx, by, bz);
        }
    }
}

/* Derivatives of the block with respect to the centres A and B:
 * d/dA_x chi_a = 2 ea chi_{a+1x} - a_x chi_{a-1x} (same for B).
 * dA[d*na*nb + ...], dB likewise; d/dC = -(d/dA + d/dB). */
void or_prim_block_deriv(int la, int lb, const double *A, double ea, const double *B, double eb,
                         const double *C, double zeta, double *dA, double *dB) {
    os_table T;
    os_build(la + lb + 1, A, ea, B, eb, C, zeta, &T);
    int na = ncart(la), nb = ncart(lb);
    for (int i = 0; i < na; ++i) {
        int a[3];
        cart(la, i, &a[0], &a[1], &a[2]);
        for (int j = 0; j < nb; ++j) {
            int b[3];
            cart(lb, j, &b[0], &b[1], &b[2]);
            for (int d = 0; d < 3; ++d) {
                int ap[3] = {a[0], a[1], a[2]}, am[3] = {a[0], a[1], a[2]};
                ap[d] += 1; am[d] -= 1;
                double va = 2.0 * ea * os_hrr(&T, ap[0], ap[1], ap[2], b[0], b[1], b[2]);
                if (a[d] > 0) va -= a[d] * os_hrr(&T, am[0], am[1], am[2], b[0], b[1], b[2]);
                int bp[3] = {b[0], b[1], b[2]}, bm[3] = {b[0], b[1], b[2]};
                bp[d] += 1; bm[d] -= 1;
                double vb = 2.0 * eb * os_hrr(&T, a[0], a[1], a[2], bp[0], bp[1], bp[2]);
                if (b[d] > 0) vb -= b[d] * os_hrr(&T, a[0], a[1], a[2], bm[0], bm[1], bm[2]);
                dA[(d * na + i) * nb + j] = va;
                dB[(d * na + i) * nb + j] = vb;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Basis normalisation (Eqs. 11-12): each Cartesian component of a           */
/* contracted shell is normalised to unit self-overlap.                      */
/* cn[cn_off[s] + comp*nprim + i] = d_i N_i(comp) / sqrt(<phi|phi>)          */
/* ------------------------------------------------------------------------ */
void or_norm_coefs(int ns, const int *sl, const int *snp, const int *soff, const double *pexp,
                   const double *pcoef, const int *cn_off, double *cn) {
    for (int s = 0; s < ns; ++s) {
        int l = sl[s], np = snp[s];
        for (int c = 0; c < ncart(l); ++c) {
            int ax, ay, az;
            cart(l, c, &ax, &ay, &az);
            double df = dfact_odd(ax) * dfact_odd(ay) * dfact_odd(az);
            double tmp[64];
            for (int i = 0; i < np; ++i) {
                double a = pexp[soff[s] + i];
                double N = sqrt(pow(2.0 * a / M_PI, 1.5) * pow(4.0 * a, l) / df);
                tmp[i] = pcoef[soff[s] + i] * N;
            }
            double ov = 0.0;
            for (int i = 0; i < np; ++i)
                for (int j = 0; j < np; ++j) {
                    double p = pexp[soff[s] + i] + pexp[soff[s] + j];
                    ov += tmp[i] * tmp[j] * pow(M_PI / p, 1.5) * df / pow(2.0 * p, l);
                }
            double sc = 1.0 / sqrt(ov);
            for (int i = 0; i < np; ++i) cn[cn_off[s] + c * np + i] = tmp[i] * sc;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Surface (Sec. 2, Eqs. 3, 7, 9; Sec. 3): r = R_I + rho_I u_j,               */
/* zeta = zeta0/(rho_I sqrt(w_j)), S = prod_{J != I} S_wf, keep if S >= thr, */
/* A_kk = diag_const * zeta / S.  S_wf written as the equal erfc form         */
/* 1/2 [erfc(z(R_J-d)) + erfc(z(R_J+d))] to avoid cancellation.              */
/* ------------------------------------------------------------------------ */
int or_surface(int N, const double *xyz, const double *rad, int ns, const double *dirs, const double *w,
               double zeta0, double thresh, double diag_const, double *r, double *zeta, double *S,
               double *Akk, int *keep) {
    int nkeep = 0;
    for (int I = 0; I < N; ++I)
        for (int j = 0; j < ns; ++j) {
            int k = I * ns + j;
            double z = zeta0 / (rad[I] * sqrt(w[j]));
            double p[3];
            for (int d = 0; d < 3; ++d) p[d] = xyz[3 * I + d] + rad[I] * dirs[3 * j + d];
            double s = 1.0;
            for (int J = 0; J < N; ++J) {
                if (J == I) continue;
                double dx = p[0] - xyz[3 * J], dy = p[1] - xyz[3 * J + 1], dz = p[2] - xyz[3 * J + 2];
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                s *= 0.5 * (erfc(z * (rad[J] - d)) + erfc(z * (rad[J] + d)));
            }
            for (int d = 0; d < 3; ++d) r[3 * k + d] = p[d];
            zeta[k] = z;
            S[k] = s;
            keep[k] = s >= thresh;
            Akk[k] = diag_const * z / s;
            nkeep += keep[k];
        }
    return nkeep;
}

/* ------------------------------------------------------------------------ */
/* Screened primitive-pair list (Sec. 4a, Eq. 15; Eq. 18 when P is given).    */
/* Bound: |c_i c_j| sqrt(2 pi^(5/2) / (p^2 sqrt(2p))) exp(-ea eb/p |A-B|^2),  */
/* with c the normalised coefficient of the x^l component.  With P, the bound */
/* is multiplied by max |P_mu nu| over the shell-pair block.                  */
/* Order: class ss, sp, sd, pp, pd, dd; shell pair (a,b) with l_a <= l_b      */
/* (a <= b when equal); primitive i of a, j of b.  weight 2 for a != b.       */
/* Returns the count; fills the arrays when out_cls != NULL.                  */
/* ------------------------------------------------------------------------ */
static const int CLS_LA[6] = {0, 0, 0, 1, 1, 2};
static const int CLS_LB[6] = {0, 1, 2, 1, 2, 2};

long or_pairs(int ns, const int *sl, const int *snp, const int *soff, const int *satom, const double *pexp,
              const int *cn_off, const double *cn, const double *xyz, const int *bf_off, int nbf,
              const double *P, double thresh, int *out_cls, int *out_a, int *out_b, int *out_i, int *out_j,
              double *out_w) {
    long n = 0;
    const double c2 = 2.0 * pow(M_PI, 2.5);
    for (int cls = 0; cls < 6; ++cls)
        for (int a = 0; a < ns; ++a) {
            if (sl[a] != CLS_LA[cls]) continue;
            for (int b = 0; b < ns; ++b) {
                if (sl[b] != CLS_LB[cls]) continue;
                if (sl[a] == sl[b] && b < a) continue;
                double pm = 1.0;
                if (P) {
                    pm = 0.0;
                    for (int mu = 0; mu < ncart(sl[a]); ++mu)
                        for (int nu = 0; nu < ncart(sl[b]); ++nu) {
                            double v = fabs(P[(long)(bf_off[a] + mu) * nbf + bf_off[b] + nu]);
                            if (v > pm) pm = v;
                        }
                }
                const double *A = xyz + 3 * satom[a], *B = xyz + 3 * satom[b];
                double ab2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
                for (int i = 0; i < snp[a]; ++i)
                    for (int j = 0; j < snp[b]; ++j) {
                        double ea = pexp[soff[a] + i], eb = pexp[soff[b] + j], p = ea + eb;
                        double ci = fabs(cn[cn_off[a] + i]), cj = fabs(cn[cn_off[b] + j]);
                        double bound = ci * cj * sqrt(c2 / (p * p * sqrt(2.0 * p))) * exp(-ea * eb / p * ab2);
                        if (pm * bound >= thresh) {
                            if (out_cls) {
                                out_cls[n] = cls; out_a[n] = a; out_b[n] = b; out_i[n] = i; out_j[n] = j;
                                out_w[n] = (a == b) ? 1.0 : 2.0;
                            }
                            ++n;
                        }
                    }
            }
        }
    return n;
}

/* common description of a molecule's basis for the integral sums */
typedef struct {
    const int *sl, *snp, *soff, *satom, *cn_off, *bf_off;
    const double *pexp, *cn, *xyz;
    int nbf;
} basis_view;

/* sum over mu in a, nu in b of X[mu,nu] c_mu_i c_nu_j blk[mu,nu] */
static double contract_block(const basis_view *bv, int a, int b, int i, int j, const double *X,
                             const double *blk) {
    int na = ncart(bv->sl[a]), nb = ncart(bv->sl[b]);
    int npa = bv->snp[a], npb = bv->snp[b];
    double s = 0.0;
    for (int mu = 0; mu < na; ++mu) {
        double cmu = bv->cn[bv->cn_off[a] + mu * npa + i];
        for (int nu = 0; nu < nb; ++nu) {
            double cnu = bv->cn[bv->cn_off[b] + nu * npb + j];
            s += X[(long)(bv->bf_off[a] + mu) * bv->nbf + bv->bf_off[b] + nu] * cmu * cnu * blk[mu * nb + nu];
        }
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* c_k = sum_{mu nu} P_{mu nu} L^k_{mu nu}, L = -(mu|J_k|nu)  (Eqs. 5, 6, 12) */
/* for the points listed in kidx (all points when kidx == NULL).              */
/* ------------------------------------------------------------------------ */
void or_esp(int ns, const int *sl, const int *snp, const int *soff, const int *satom, const double *pexp,
            const int *cn_off, const double *cn, const double *xyz, const int *bf_off, int nbf,
            const double *P, long npairs, const int *pa, const int *pb, const int *pi, const int *pj,
            const double *pw, int npts, const double *r, const double *zeta, int nk, const int *kidx,
            double *c_out) {
    basis_view bv = {sl, snp, soff, satom, cn_off, bf_off, pexp, cn, xyz, nbf};
    (void)ns; (void)npts;
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < nk; ++t) {
        int k = kidx ? kidx[t] : t;
        double acc = 0.0, blk[36];
        for (long q = 0; q < npairs; ++q) {
            int a = pa[q], b = pb[q];
            or_prim_block(sl[a], sl[b], xyz + 3 * satom[a], pexp[soff[a] + pi[q]], xyz + 3 * satom[b],
                          pexp[soff[b] + pj[q]], r + 3 * k, zeta[k], blk);
            acc -= pw[q] * contract_block(&bv, a, b, pi[q], pj[q], P, blk);
        }
        c_out[t] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Fock correction F_{mu nu} += sum_k q_k L^k_{mu nu}  (Eqs. 10, 16, 17).     */
/* Pairs must be grouped by shell pair (as or_pairs emits them); when sp_sel  */
/* is given only shell pairs with sp_sel[a*ns+b] != 0 are done.  Blocks are   */
/* written for (a,b) and, for a != b, mirrored to (b,a).                      */
/* ------------------------------------------------------------------------ */
void or_fock(int ns, const int *sl, const int *snp, const int *soff, const int *satom, const double *pexp,
             const int *cn_off, const double *cn, const double *xyz, const int *bf_off, int nbf,
             long npairs, const int *pa, const int *pb, const int *pi, const int *pj, int npts,
             const double *r, const double *zeta, const double *q, const unsigned char *sp_sel, double *F) {
    /* shell-pair group boundaries */
    long ngroups = 0;
    long *gstart = (long *)malloc(sizeof(long) * (npairs + 1));
    for (long t = 0; t < npairs; ++t)
        if (t == 0 || pa[t] != pa[t - 1] || pb[t] != pb[t - 1]) gstart[ngroups++] = t;
    gstart[ngroups] = npairs;
#pragma omp parallel for schedule(dynamic, 1)
    for (long g = 0; g < ngroups; ++g) {
        int a = pa[gstart[g]], b = pb[gstart[g]];
        if (sp_sel && !sp_sel[(long)a * ns + b]) continue;
        int la = sl[a], lb = sl[b], na = ncart(la), nb = ncart(lb);
        double acc[36], blk[36];
        memset(acc, 0, sizeof(acc));
        for (long t = gstart[g]; t < gstart[g + 1]; ++t) {
            int i = pi[t], j = pj[t];
            for (int k = 0; k < npts; ++k) {
                or_prim_block(la, lb, xyz + 3 * satom[a], pexp[soff[a] + i], xyz + 3 * satom[b],
                              pexp[soff[b] + j], r + 3 * k, zeta[k], blk);
                for (int mu = 0; mu < na; ++mu)
                    for (int nu = 0; nu < nb; ++nu)
                        acc[mu * nb + nu] -= q[k] * cn[cn_off[a] + mu * snp[a] + i] * cn[cn_off[b] + nu * snp[b] + j] *
                                             blk[mu * nb + nu];
            }
        }
        for (int mu = 0; mu < na; ++mu)
            for (int nu = 0; nu < nb; ++nu) {
                F[(long)(bf_off[a] + mu) * nbf + bf_off[b] + nu] += acc[mu * nb + nu];
                if (a != b) F[(long)(bf_off[b] + nu) * nbf + bf_off[a] + mu] += acc[mu * nb + nu];
            }
    }
    free(gstart);
}

/* ------------------------------------------------------------------------ */
/* A and B (Sec. 2, Eqs. 2, 3, 4, 8).  Coincident positions take the limit   */
/* 2 z / sqrt(pi).                                                           */
/* ------------------------------------------------------------------------ */
static double a_offdiag(const double *rk, double zk, const double *rl, double zl) {
    double zp = zk * zl / sqrt(zk * zk + zl * zl);
    double dx = rk[0] - rl[0], dy = rk[1] - rl[1], dz = rk[2] - rl[2];
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (d == 0.0) return 2.0 * zp / sqrt(M_PI);
    return erf(zp * d) / d;
}

void or_amat(int M, const double *r, const double *zeta, const double *Akk, double *A) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < M; ++k)
        for (int l = 0; l < M; ++l)
            A[(long)k * M + l] = (k == l) ? Akk[k] : a_offdiag(r + 3 * k, zeta[k], r + 3 * l, zeta[l]);
}

void or_arow(int M, int k, const double *r, const double *zeta, const double *Akk, double *row) {
    for (int l = 0; l < M; ++l) row[l] = (k == l) ? Akk[k] : a_offdiag(r + 3 * k, zeta[k], r + 3 * l, zeta[l]);
}

/* y = A x for the rows listed in kidx (all rows when kidx == NULL) */
void or_matvec(int M, const double *r, const double *zeta, const double *Akk, const double *x, int nk,
               const int *kidx, double *y) {
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nk; ++t) {
        int k = kidx ? kidx[t] : t;
        double s = 0.0;
        for (int l = 0; l < M; ++l)
            s += ((k == l) ? Akk[k] : a_offdiag(r + 3 * k, zeta[k], r + 3 * l, zeta[l])) * x[l];
        y[t] = s;
    }
}

void or_bz(int M, const double *r, const double *zeta, int N, const double *xyz, const double *Z, double *out) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < M; ++k) {
        double s = 0.0;
        for (int J = 0; J < N; ++J) {
            double dx = r[3 * k] - xyz[3 * J], dy = r[3 * k + 1] - xyz[3 * J + 1], dz = r[3 * k + 2] - xyz[3 * J + 2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            s += Z[J] * (d == 0.0 ? 2.0 * zeta[k] / sqrt(M_PI) : erf(zeta[k] * d) / d);
        }
        out[k] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Gradient at fixed density (Sec. 2, Eq. 14; Sec. 4c, Eq. 22).               */
/* Outputs, per term t (0: B, 1: c, 2: A off-diagonal, 3: A diagonal):       */
/*   gn[t*3N + 3I + d]  partial derivative w.r.t. nucleus I (points fixed)   */
/*   gs[t*3M + 3k + d]  partial derivative w.r.t. surface point k            */
/* The c-term sign follows L = -(mu|J|nu); the operator-centre derivative is */
/* -(d/dA + d/dB) by translation invariance.                                  */
/* ------------------------------------------------------------------------ */
static double dg_erf(double z, double d) { /* d/dd [erf(z d)/d] */
    return 2.0 * z / sqrt(M_PI) * exp(-z * z * d * d) / d - erf(z * d) / (d * d);
}

/* all four terms for one surface point k: gsk[t*3 + d] (point side) and, when gnl is
 * given, the nucleus-side contributions accumulated into gnl[t*3N + 3J + d] */
static void grad_point(const basis_view *bv, const double *Zn, const double *rad, int N, const double *P,
                       long npairs, const int *pa, const int *pb, const int *pi, const int *pj, const double *pw,
                       int M, const double *r, const double *zeta, const double *Akk, const int *owner,
                       const double *q, double f, int k, double *gsk, double *gnl) {
    const int *sl = bv->sl, *soff = bv->soff, *satom = bv->satom;
    const double *pexp = bv->pexp, *xyz = bv->xyz;
    const double *rk = r + 3 * k;
    memset(gsk, 0, sizeof(double) * 12);
    /* term 0: q_k z_J d/dx erf(zeta_k d)/d */
    for (int J = 0; J < N; ++J) {
        double v[3] = {rk[0] - xyz[3 * J], rk[1] - xyz[3 * J + 1], rk[2] - xyz[3 * J + 2]};
        double d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (d == 0.0) continue;
        double g = q[k] * Zn[J] * dg_erf(zeta[k], d) / d;
        for (int e = 0; e < 3; ++e) {
            gsk[e] += g * v[e];
            if (gnl) gnl[3 * J + e] -= g * v[e];
        }
    }
    /* term 1: q_k d c_k */
    double dA[3 * 36], dB[3 * 36];
    for (long t = 0; t < npairs; ++t) {
        int a = pa[t], b = pb[t];
        or_prim_block_deriv(sl[a], sl[b], xyz + 3 * satom[a], pexp[soff[a] + pi[t]], xyz + 3 * satom[b],
                            pexp[soff[b] + pj[t]], rk, zeta[k], dA, dB);
        int nn = ncart(sl[a]) * ncart(sl[b]);
        for (int e = 0; e < 3; ++e) {
            double ga = -pw[t] * q[k] * contract_block(bv, a, b, pi[t], pj[t], P, dA + e * nn);
            double gb = -pw[t] * q[k] * contract_block(bv, a, b, pi[t], pj[t], P, dB + e * nn);
            if (gnl) {
                gnl[3 * N + 3 * satom[a] + e] += ga;
                gnl[3 * N + 3 * satom[b] + e] += gb;
            }
            gsk[3 + e] -= ga + gb;
        }
    }
    /* term 2: (1/2f) q^T dA_off q, d/dr_k picks up both A_kl and A_lk */
    for (int l = 0; l < M; ++l) {
        if (l == k) continue;
        const double *rl = r + 3 * l;
        double v[3] = {rk[0] - rl[0], rk[1] - rl[1], rk[2] - rl[2]};
        double d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (d == 0.0) continue;
        double zp = zeta[k] * zeta[l] / sqrt(zeta[k] * zeta[k] + zeta[l] * zeta[l]);
        double g = q[k] * q[l] / f * dg_erf(zp, d) / d;
        for (int e = 0; e < 3; ++e) gsk[6 + e] += g * v[e];
    }
    /* term 3: (1/2f) q_k^2 dA_kk, A_kk = const zeta / prod S_wf */
    int I = owner[k];
    double zk = zeta[k];
    for (int J = 0; J < N; ++J) {
        if (J == I) continue;
        double v[3] = {rk[0] - xyz[3 * J], rk[1] - xyz[3 * J + 1], rk[2] - xyz[3 * J + 2]};
        double d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (d == 0.0) continue;
        double sw = 0.5 * (erfc(zk * (rad[J] - d)) + erfc(zk * (rad[J] + d)));
        double dsw = zk / sqrt(M_PI) *
                     (exp(-zk * zk * (rad[J] - d) * (rad[J] - d)) - exp(-zk * zk * (rad[J] + d) * (rad[J] + d)));
        double g = 0.5 / f * q[k] * q[k] * (-Akk[k]) * dsw / sw / d;
        for (int e = 0; e < 3; ++e) {
            gsk[9 + e] += g * v[e];
            if (gnl) gnl[3 * 3 * N + 3 * J + e] -= g * v[e];
        }
    }
}

void or_grad(int ns, const int *sl, const int *snp, const int *soff, const int *satom, const double *pexp,
             const int *cn_off, const double *cn, const double *xyz, const int *bf_off, int nbf, const double *Zn,
             const double *rad, int N, const double *P, long npairs, const int *pa, const int *pb, const int *pi,
             const int *pj, const double *pw, int M, const double *r, const double *zeta, const double *Akk,
             const int *owner, const double *q, double f, double *gn, double *gs) {
    basis_view bv = {sl, snp, soff, satom, cn_off, bf_off, pexp, cn, xyz, nbf};
    (void)ns;
    memset(gn, 0, sizeof(double) * 4 * 3 * N);
    memset(gs, 0, sizeof(double) * 4 * 3 * M);
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *gn_thr = (double *)calloc((size_t)nthr * 4 * 3 * N, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gnl = gn_thr + (size_t)tid * 4 * 3 * N;
        double gsk[12];
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < M; ++k) {
            grad_point(&bv, Zn, rad, N, P, npairs, pa, pb, pi, pj, pw, M, r, zeta, Akk, owner, q, f, k, gsk, gnl);
            for (int t = 0; t < 4; ++t)
                for (int e = 0; e < 3; ++e) gs[t * 3 * M + 3 * k + e] = gsk[3 * t + e];
        }
    }
    for (int t = 0; t < nthr; ++t)
        for (int i = 0; i < 4 * 3 * N; ++i) gn[i] += gn_thr[(size_t)t * 4 * 3 * N + i];
    free(gn_thr);
}

/* surface-point gradient (sum of the four terms) for the points listed in kidx only */
void or_grad_points(int ns, const int *sl, const int *snp, const int *soff, const int *satom, const double *pexp,
                    const int *cn_off, const double *cn, const double *xyz, const int *bf_off, int nbf,
                    const double *Zn, const double *rad, int N, const double *P, long npairs, const int *pa,
                    const int *pb, const int *pi, const int *pj, const double *pw, int M, const double *r,
                    const double *zeta, const double *Akk, const int *owner, const double *q, double f, int nk,
                    const int *kidx, double *gs_out) {
    basis_view bv = {sl, snp, soff, satom, cn_off, bf_off, pexp, cn, xyz, nbf};
    (void)ns;
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < nk; ++t) {
        double gsk[12];
        grad_point(&bv, Zn, rad, N, P, npairs, pa, pb, pi, pj, pw, M, r, zeta, Akk, owner, q, f, kidx[t], gsk, NULL);
        for (int e = 0; e < 3; ++e) gs_out[3 * t + e] = gsk[e] + gsk[3 + e] + gsk[6 + e] + gsk[9 + e];
    }
}

/* ------------------------------------------------------------------------ */
/* Randomized block-Jacobi partition (Sec. 4b-ii).  SplitMix64 stream; the   */
/* unassigned indices are kept ascending; pivot = list[floor(u n_left)] with */
/* u = (x >> 11) 2^-53; the block is the pivot plus the l-1 unassigned       */
/* indices of largest |A_kl| (ties: smaller index first); members are stored */
/* ascending.  Returns the number of blocks.                                 */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct { double v; int i; } rank_t;

static int rank_cmp(const void *x, const void *y) {
    const rank_t *a = (const rank_t *)x, *b = (const rank_t *)y;
    if (a->v > b->v) return -1;
    if (a->v < b->v) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

static int int_cmp(const void *x, const void *y) {
    int a = *(const int *)x, b = *(const int *)y;
    return (a > b) - (a < b);
}

int or_rbj_partition(int M, const double *r, const double *zeta, int l, uint64_t seed, int *perm, int *blk_off) {
    int *left = (int *)malloc(sizeof(int) * M);
    rank_t *rk = (rank_t *)malloc(sizeof(rank_t) * M);
    unsigned char *take = (unsigned char *)calloc(M, 1);
    for (int i = 0; i < M; ++i) left[i] = i;
    int n_left = M, nb = 0, filled = 0;
    uint64_t st = seed;
    blk_off[0] = 0;
    while (n_left > 0) {
        uint64_t x = splitmix64(&st);
        double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
        int pos = (int)floor(u * (double)n_left);
        if (pos >= n_left) pos = n_left - 1;
        int piv = left[pos];
        int m = 0;
        for (int t = 0; t < n_left; ++t) {
            int c = left[t];
            if (c == piv) continue;
            rk[m].v = fabs(a_offdiag(r + 3 * piv, zeta[piv], r + 3 * c, zeta[c]));
            rk[m].i = c;
            ++m;
        }
        qsort(rk, m, sizeof(rank_t), rank_cmp);
        int take_n = (l - 1 < m) ? l - 1 : m;
        int start = filled;
        perm[filled++] = piv;
        take[piv] = 1;
        for (int t = 0; t < take_n; ++t) { perm[filled++] = rk[t].i; take[rk[t].i] = 1; }
        qsort(perm + start, filled - start, sizeof(int), int_cmp);
        int w = 0;
        for (int t = 0; t < n_left; ++t)
            if (!take[left[t]]) left[w++] = left[t];
        n_left = w;
        blk_off[++nb] = filled;
    }
    free(left); free(rk); free(take);
    return nb;
}
