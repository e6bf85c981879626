// Integral kernels of the C-PCM path on gfx950.
//
//   c_k  = sum_{mu nu} P_{mu nu} L^k_{mu nu}        (Sec. 2, Eqs. 5-6, 12)
//   F   += sum_k q_k L^k                            (Sec. 2, Eq. 10; Sec. 4a, Eqs. 16-17)
//   (Bz)_k = sum_J Z_J erf(zeta_k d)/d              (Sec. 2, Eq. 4)
//
// Each (primitive pair, point) evaluation is a Hermite (McMurchie-Davidson) expansion:
// the pair's density-contracted coefficients D_tuv (esp) or the accumulated V_tuv (Fock)
// factor out of the point loop, so an evaluation is R^(n)_000, the R_tuv build and an
// n_tuv-term dot product.
//
// Mapping.  esp: one lane per surface point; the wave walks a chunk of primitive pairs
// whose records are wave-uniform (scalar loads into SGPRs, a few pairs per batch so one
// wait covers several evaluations); the k-sum stays in a register.  Fock: one lane per
// primitive pair; the wave walks a chunk of points (wave-uniform, batches of four) and
// accumulates V_tuv in registers.  Pair lists and point arrays are padded with
// zero-contribution entries so batches never need a tail.  Partial results per chunk are
// reduced afterwards in a fixed order, so results are bitwise reproducible.
//
// Batching.  One launch per angular class covers every molecule of a batch: work items are
// (molecule, tile, chunk) triples located through per-molecule descriptors, one per
// workgroup.  Each kernel stages only the Boys-table columns its order needs, so low-L
// kernels keep more workgroups resident.  The chunk shape of each (class, size bucket) is
// chosen by timing a few candidates on first use.
#include "pcm_internal.h"
#include "low_order.h"
#include "contract.h"

#include <algorithm>
#include <array>
#include <cstring>
#include <memory>

// ----------------------------------------------------------------------------------------
// Work items.  A launch covers one class for a set of molecules; each (molecule, class) has
// a descriptor with the base index of its items, and an item index maps to (molecule, tile,
// chunk) by a binary search over the bases, so the tables stay one entry per molecule.
// ----------------------------------------------------------------------------------------
struct EspDesc {
    const unsigned char *rec;  // class records (header + D_tuv), padded to REC_PAD
    const void *pts;           // PtInt<T> [Mpad]
    const int *pperm;          // point taken by each lane (null: surface order)
    double *part;              // partial rows of this molecule
    long long base;            // first item
    int M, stride, n_pad, chunk, ntile, row0;
};

struct FockDesc {
    const unsigned char *rec;  // class headers
    const int *perm;           // record taken by each lane, class-local (null: list order)
    const void *pts;           // PtInt<T> [Mpad]
    const double *q;           // charges, zero past M [Mpad]
    double *vout;              // [nch][NT][n_pairs]
    long long base;
    int n_pairs, Mpad, chunk, nptile, stride;
};

struct SumDesc {
    const double *part;
    double *out;
    long long base;
    int M, rows, acc;  // acc: add to out instead of overwriting it
};


// ----------------------------------------------------------------------------------------
// esp: partial c over one chunk of pairs of one class; lane = surface point
// ----------------------------------------------------------------------------------------
template <int L, typename T, typename B>
__global__ __launch_bounds__(256) void k_esp(const EspDesc *__restrict__ ds, int nd, long long n_items,
                                             const B *__restrict__ boys_g) {
    constexpr int NT = ntuv(L), PB = pair_batch<L>();
    __shared__ B tab[boys_lds_size<B, L>()];
    load_boys<B, L>(tab, boys_g);
    for (long long it = blockIdx.x; it < n_items; it += gridDim.x) {
        const EspDesc &d = ds[find_desc(ds, nd, it)];
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
        double acc = 0.0;
        for (int ip = p0; ip < p1; ip += PB) {
            PairHdr<T> h[PB];
            T D[PB][NT];
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const cptr<unsigned char> r = rec + (size_t)(ip + b) * stride;
                h[b] = *(cptr<PairHdr<T>>)(r);
                const cptr<T> dd = (cptr<T>)(r + sizeof(PairHdr<T>));
#pragma unroll
                for (int t = 0; t < NT; ++t) D[b][t] = dd[t];
            }
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                if constexpr (L == 3) {
                    // sum_t D_t R_t = D_0 R^(0) + lin R^(1) + quad R^(2) + C R^(3): quad holds the
                    // second-order terms and the first-order parts of the third-order R_tuv, C the
                    // cubic form (D index 10 .. 19: 300, 210, 201, 120, 111, 102, 030, 021, 012, 003)
                    const T *Db = D[b];
                    T x, y, z, Rn[4];
                    eval_Rn<3, T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim,
                                  tab, x, y, z, Rn);
                    const T zz = z * z, three = T(3);
                    const T lin = fma(Db[1], x, fma(Db[2], y, fma(Db[3], z, Db[4] + Db[7] + Db[9])));
                    const T bx = fma(three, Db[10], Db[13] + Db[15]);
                    const T by = fma(three, Db[16], Db[11] + Db[18]);
                    const T bz = fma(three, Db[19], Db[12] + Db[17]);
                    const T quad = fma(x, fma(Db[4], x, fma(Db[5], y, fma(Db[6], z, bx))),
                                       fma(y, fma(Db[7], y, fma(Db[8], z, by)), z * fma(Db[9], z, bz)));
                    const T cub = fma(x, fma(x, fma(Db[10], x, fma(Db[11], y, Db[12] * z)),
                                             fma(y, fma(Db[13], y, Db[14] * z), Db[15] * zz)),
                                      fma(y, fma(y, fma(Db[16], y, Db[17] * z), Db[18] * zz), Db[19] * zz * z));
                    if constexpr (sizeof(T) == 8) {
                        acc = fma(Db[0], Rn[0], acc);
                        acc = fma(lin, Rn[1], acc);
                        acc = fma(quad, Rn[2], acc);
                        acc = fma(cub, Rn[3], acc);
                    } else {
                        acc += (double)fma(cub, Rn[3], fma(quad, Rn[2], fma(lin, Rn[1], Db[0] * Rn[0])));
                    }
                    continue;
                }
                if constexpr (L == 2) {
                    // sum_t D_t R_t = D_0 R^(0) + R^(1) (D_100 X + D_010 Y + D_001 Z + D_200 + D_020 + D_002)
                    //               + R^(2) (the quadratic form of D_200 ... D_002 in X, Y, Z)
                    const T *Db = D[b];
                    T x, y, z, Rn[3];
                    eval_Rn<2, T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim,
                                  tab, x, y, z, Rn);
                    const T q1 = fma(Db[4], x, fma(Db[5], y, Db[6] * z));
                    const T q2 = fma(Db[7], y, Db[8] * z);
                    const T qf = fma(x, q1, fma(y, q2, z * (Db[9] * z)));
                    const T lin = fma(Db[1], x, fma(Db[2], y, fma(Db[3], z, Db[4] + Db[7] + Db[9])));
                    if constexpr (sizeof(T) == 8) {
                        acc = fma(Db[0], Rn[0], acc);
                        acc = fma(lin, Rn[1], acc);
                        acc = fma(qf, Rn[2], acc);
                    } else {  // FP32 evaluation, one FP64 add per pair
                        acc += (double)fma(qf, Rn[2], fma(lin, Rn[1], Db[0] * Rn[0]));
                    }
                    continue;
                }
                if constexpr (L == 1) {  // sum_t D_t R_t with R^(1) factored out
                    T x, y, z, Rn[2];
                    eval_Rn1<T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim, tab,
                                x, y, z, Rn);
                    const T w = fma(D[b][1], x, fma(D[b][2], y, D[b][3] * z));
                    if constexpr (sizeof(T) == 8) {
                        acc = fma(D[b][0], Rn[0], acc);
                        acc = fma(w, Rn[1], acc);
                    } else {
                        acc += (double)fma(w, Rn[1], D[b][0] * Rn[0]);
                    }
                    continue;
                }
                T R[NT];
                eval_R<L, T, B>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim, tab,
                             R);
                if constexpr (sizeof(T) == 8) {  // FP64: straight into the accumulator
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc = fma(D[b][t], R[t], acc);
                } else {  // FP32 evaluation, one FP64 add per pair
                    T s = T(0);
#pragma unroll
                    for (int t = 0; t < NT; ++t) s = fma(D[b][t], R[t], s);
                    acc += (double)s;
                }
            }
        }
        if (k < M) d.part[(size_t)(d.row0 + ch) * M + kk] = acc;
    }
}

// fixed-order sum of partial rows: out[k] = sum_r part[r*M + k]; item = 256 points
__global__ __launch_bounds__(256) void k_sum_rows(const SumDesc *__restrict__ ds, int nd, long long n_items) {
    for (long long it = blockIdx.x; it < n_items; it += gridDim.x) {
        const SumDesc &d = ds[find_desc(ds, nd, it)];
        const int k = (int)(it - d.base) * 256 + threadIdx.x;
        if (k >= d.M) continue;
        double s = 0.0;
        for (int r = 0; r < d.rows; ++r) s += d.part[(size_t)r * d.M + k];
        d.out[k] = d.acc ? d.out[k] + s : s;
    }
}

// ----------------------------------------------------------------------------------------
// Bz (Eq. 4); coincident positions take the limit 2 zeta / sqrt(pi)
// ----------------------------------------------------------------------------------------
__global__ void k_bz(const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ pz,
                     int M, const double *__restrict__ zeta, const double *__restrict__ xyz,
                     const double *__restrict__ Z, int N, double *__restrict__ bz) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double x = px[k], y = py[k], z = pz[k], zk = zeta[k];
    double s = 0.0;
    for (int J = 0; J < N; ++J) {
        double dx = x - xyz[3 * J], dy = y - xyz[3 * J + 1], dz = z - xyz[3 * J + 2];
        double d2 = dx * dx + dy * dy + dz * dz;
        double v;
        if (d2 == 0.0) {
            v = 2.0 * zk * 0.56418958354775628695;  // 2 zeta / sqrt(pi)
        } else {
            double d = sqrt(d2);
            v = (zk * d >= 6.0) ? 1.0 / d : erf(zk * d) / d;
        }
        s += Z[J] * v;
    }
    bz[k] = s;
}

void bz_launches(pcm_ctx *ctx, pcm_mol *mol, double *bz, Launches &out) {
    const int M = mol->M, N = mol->N;
    const double *px = mol->px.p, *py = mol->py.p, *pz = mol->pz.p, *zeta = mol->zeta.p, *xyz = mol->xyz.p,
                 *Z = mol->Z.p;
    out.add("bz", (double)M * N, [=](hipStream_t st) {
        k_bz<<<grid_for(M, 256), 256, 0, st>>>(px, py, pz, M, zeta, xyz, Z, N, bz);
        HIP_LAUNCH_OK();
    });
}

void run_bz(pcm_ctx *ctx, pcm_mol *mol, double *bz) {
    ProfScope ps(ctx, "bz", (double)mol->M * mol->N);
    k_bz<<<grid_for(mol->M, 256), 256, 0, ctx->stream>>>(mol->px.p, mol->py.p, mol->pz.p, mol->M, mol->zeta.p,
                                                          mol->xyz.p, mol->Z.p, mol->N, bz);
    HIP_LAUNCH_OK();
}

// ----------------------------------------------------------------------------------------
// Fock: V_tuv(pair) = sum_k q_k R_tuv(pair, k) over one chunk of points; lane = primitive pair
// ----------------------------------------------------------------------------------------
template <int L, typename T, typename B>
__global__ __launch_bounds__(256) void k_fock_v(const FockDesc *__restrict__ ds, int nd, long long n_items,
                                                const B *__restrict__ boys_g) {
    constexpr int NT = ntuv(L);
    __shared__ B tab[boys_lds_size<B, L>()];
    load_boys<B, L>(tab, boys_g);
    for (long long it = blockIdx.x; it < n_items; it += gridDim.x) {
        const FockDesc &d = ds[find_desc(ds, nd, it)];
        const long long local = it - d.base;
        const int pt_tile = (int)(local % d.nptile), ch = (int)(local / d.nptile);
        const int n = d.n_pairs;
        const int ip = pt_tile * 256 + threadIdx.x;
        const int ipp = d.perm ? d.perm[ip < n ? ip : n - 1] : (ip < n ? ip : n - 1);
        const PairHdr<T> h = *reinterpret_cast<const PairHdr<T> *>(d.rec + (size_t)ipp * d.stride);
        const cptr<PtInt<T>> pts = as_const(reinterpret_cast<const PtInt<T> *>(d.pts));
        const cptr<double> q = as_const(d.q);
        const int k0 = ch * d.chunk;
        const int k1 = min(d.Mpad, k0 + d.chunk);
        double V[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) V[t] = 0.0;
        // FP64 records (V up to order 1 .. 4): the far-field factored sums of low_order.h
        constexpr bool FS = sizeof(T) == 8 && L >= 1;
        constexpr int NS = FS ? L : 2;  // L = 0 (V_000 alone) keeps its plain form
        double S[nsums<NS>()], ipf = 0.0;
        if constexpr (FS) {
#pragma unroll
            for (int t = 0; t < nsums<NS>(); ++t) S[t] = 0.0;
            ipf = far_scale(h.pf);
        }
        for (int k = k0; k < k1; k += PT_BATCH) {
            PtInt<T> pt[PT_BATCH];
            double qk[PT_BATCH];
#pragma unroll
            for (int b = 0; b < PT_BATCH; ++b) {
                pt[b] = pts[k + b];
                qk[b] = q[k + b];
            }
#pragma unroll
            for (int b = 0; b < PT_BATCH; ++b) {
                if constexpr (FS) {
                    double x, y, z, sv[NS + 1];
                    eval_s<NS, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, ipf, pt[b].zeta2, pt[b].zeta,
                                  pt[b].lim, tab, qk[b], x, y, z, sv);
                    acc_S<NS>(sv, x, y, z, S);
                    continue;
                }
                if constexpr (L == 2) {  // q R_t with q R^(1), q R^(2) formed once
                    T x, y, z, Rn[3];
                    eval_Rn<2, T, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta,
                                  pt[b].lim, tab, x, y, z, Rn);
                    acc_V2<T>(qk[b], x, y, z, Rn, V);
                    continue;
                }
                if constexpr (L == 3) {  // q R_t with q R^(1..3) formed once
                    T x, y, z, Rn[4];
                    eval_Rn<3, T, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta,
                                  pt[b].lim, tab, x, y, z, Rn);
                    acc_V3<T>(qk[b], x, y, z, Rn, V);
                    continue;
                }
                if constexpr (L == 1) {  // q R_t with q R^(1) formed once
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
                eval_R<L, T, B>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta, pt[b].lim,
                             tab, R);
#pragma unroll
                for (int t = 0; t < NT; ++t) V[t] = fma(qk[b], (double)R[t], V[t]);
            }
        }
        if constexpr (FS) fin_S<NS>(h.pf, S, V);
        if (ip < n) {
            double *o = d.vout + (size_t)ch * NT * n;
#pragma unroll
            for (int t = 0; t < NT; ++t) o[(size_t)t * n + ip] = V[t];
        }
    }
}

// Contraction and scatter of one class for every molecule of a call: one descriptor per
// molecule; contraction items are primitive pairs (from `base`), scatter items candidate shell
// pairs (from `sbase`).
struct FockCDesc {
    long long base, sbase;   // first contraction / scatter item of this molecule
    long long n, nsp;        // primitive pairs of the class, candidate shell pairs of the class
    long long sp0, cls_off;  // first candidate shell pair, offset of the class in the list
    int nch, nbf;
    int vnt;                          // V entries per (chunk, pair): ntuv(L), or ntuv(L+1) for V' of the gradient
    const unsigned long long *memb;   // null, or per candidate shell pair the bits of this term's list: an
                                      // entry of a merged list without its bit gets a zero block
    const double *vin;                // V by slot of the pair order (vperm), else by list entry
    const int *vperm;                 // slot -> class-local list entry (null: the identity)
    const int *es, *ei, *spo, *spa, *spb, *snp, *soff, *satom, *cnoff, *bfo;
    const double *pexp, *cn, *xyz;
    double *fprim, *F;
};

__device__ __forceinline__ int find_sdesc(const FockCDesc *__restrict__ ds, int nd, long long it) {
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (ds[mid].sbase <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// per primitive pair: F_prim[mu nu] = -c_mu_i c_nu_j sum_tuv E^{mu nu}_tuv V_tuv
template <int LA, int LB>
__global__ void k_fock_contract(const FockCDesc *__restrict__ ds, int nd, long long total) {
    constexpr int L = LA + LB, NT = ntuv(L), NC = ncart(LA) * ncart(LB);
    const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= total) return;
    const FockCDesc &d = ds[find_desc(ds, nd, it)];
    const long long qs = it - d.base, n = d.n;  // slot of the pair order
    const long long q = d.vperm ? d.vperm[qs] : qs;
    int sp = d.es[q], ij = d.ei[q];
    if (d.memb && !((d.memb[sp] >> ij) & 1ull)) {
        for (int c = 0; c < NC; ++c) d.fprim[(size_t)q * NC + c] = 0.0;
        return;
    }
    // sums over the chunks in chunk order; the loads of one chunk are issued together
    double V[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) V[t] = 0.0;
    for (int c = 0; c < d.nch; ++c) {
        const double *__restrict__ vc = d.vin + (size_t)c * d.vnt * n + qs;
        double u[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) u[t] = vc[(size_t)t * n];
#pragma unroll
        for (int t = 0; t < NT; ++t) V[t] += u[t];
    }
    int a = d.spa[sp], b = d.spb[sp], i = ij >> 3, j = ij & 7;
    double ea = d.pexp[d.soff[a] + i], eb = d.pexp[d.soff[b] + j], p = ea + eb;
    const double *A = d.xyz + 3 * d.satom[a], *B = d.xyz + 3 * d.satom[b];
    double P[3] = {(ea * A[0] + eb * B[0]) / p, (ea * A[1] + eb * B[1]) / p, (ea * A[2] + eb * B[2]) / p};
    Herm1D<LA, LB> ex, ey, ez;
    double inv2p = 0.5 / p;
    ex.build(P[0] - A[0], P[0] - B[0], inv2p);
    ey.build(P[1] - A[1], P[1] - B[1], inv2p);
    ez.build(P[2] - A[2], P[2] - B[2], inv2p);
    for (int mu = 0; mu < ncart(LA); ++mu) {
        int ax, ay, az;
        cart_comp(LA, mu, ax, ay, az);
        double cmu = d.cn[d.cnoff[a] + mu * d.snp[a] + i];
        for (int nu = 0; nu < ncart(LB); ++nu) {
            int bx, by, bz;
            cart_comp(LB, nu, bx, by, bz);
            double s = 0.0;
            for (int t = 0; t <= ax + bx; ++t)
                for (int u = 0; u <= ay + by; ++u) {
                    double etu = ex.e[ax][bx][t] * ey.e[ay][by][u];
                    for (int v = 0; v <= az + bz; ++v) s += etu * ez.e[az][bz][v] * V[tuv_idx(t, u, v)];
                }
            d.fprim[(size_t)q * NC + mu * ncart(LB) + nu] = -cmu * d.cn[d.cnoff[b] + nu * d.snp[b] + j] * s;
        }
    }
}

// The same for classes with many Cartesian products (L >= 3): one wave per primitive pair,
// V and the Hermite tables in LDS, lane mu * ncart(LB) + nu writes one product.
constexpr int FCW_WAVES = 4;
template <int LA, int LB>
__global__ __launch_bounds__(64 * FCW_WAVES) void k_fock_contract_w(const FockCDesc *__restrict__ ds, int nd,
                                                                     long long total) {
    constexpr int L = LA + LB, NT = ntuv(L), TS = LA + LB + 1, ES = herm1d_size<LA, LB>();
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = NA * NB;
    static_assert(NC <= 64, "one lane per product of Cartesian components");
    __shared__ double sV[FCW_WAVES][NT];
    __shared__ double sE[FCW_WAVES][3][ES];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long it = (long long)blockIdx.x * FCW_WAVES + w;
    const bool in_range = it < total;
    const FockCDesc &d = ds[in_range ? find_desc(ds, nd, it) : 0];
    const long long qs = it - d.base, n = d.n;  // slot of the pair order
    const long long q = in_range && d.vperm ? d.vperm[qs] : qs;
    const bool valid = in_range && (!d.memb || ((d.memb[d.es[q]] >> d.ei[q]) & 1ull));
    int a = 0, b = 0, i = 0, j = 0;
    if (valid) {
        const int sp = d.es[q], ij = d.ei[q];
        a = d.spa[sp];
        b = d.spb[sp];
        i = ij >> 3;
        j = ij & 7;
        if (lane < NT) {
            sV[w][lane] = chunk_sum(d.vin + (size_t)lane * n + qs, (size_t)d.vnt * n, d.nch);
        }
        if (lane < 3) {
            const double ea = d.pexp[d.soff[a] + i], eb = d.pexp[d.soff[b] + j], p = ea + eb;
            const double Ad = d.xyz[3 * d.satom[a] + lane], Bd = d.xyz[3 * d.satom[b] + lane];
            const double Pd = (ea * Ad + eb * Bd) / p;
            herm1d_build_lds<LA, LB>(sE[w][lane], Pd - Ad, Pd - Bd, 0.5 / p);
        }
    }
    __syncthreads();
    if (!in_range || lane >= NC) return;
    if (!valid) {
        d.fprim[(size_t)q * NC + lane] = 0.0;
        return;
    }
    const int mu = lane / NB, nu = lane - mu * NB;
    int ax, ay, az, bx, by, bz;
    cart_comp(LA, mu, ax, ay, az);
    cart_comp(LB, nu, bx, by, bz);
    const double *ex = sE[w][0], *ey = sE[w][1], *ez = sE[w][2];
    double s = 0.0;
    for (int t = 0; t <= ax + bx; ++t)
        for (int u = 0; u <= ay + by; ++u) {
            const double etu = ex[(ax * (LB + 1) + bx) * TS + t] * ey[(ay * (LB + 1) + by) * TS + u];
            for (int v = 0; v <= az + bz; ++v) s += etu * ez[(az * (LB + 1) + bz) * TS + v] * sV[w][tuv_idx(t, u, v)];
        }
    d.fprim[(size_t)q * NC + lane] = -d.cn[d.cnoff[a] + mu * d.snp[a] + i] * d.cn[d.cnoff[b] + nu * d.snp[b] + j] * s;
}

// per candidate shell pair: sum its primitive pairs in list order and add the block to F
template <int LA, int LB>
__global__ void k_fock_scatter(const FockCDesc *__restrict__ ds, int nd, long long total) {
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = NA * NB;
    const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= total) return;
    const FockCDesc &d = ds[find_sdesc(ds, nd, it)];
    const long long sp = d.sp0 + (it - d.sbase);
    int g0 = d.spo[sp], g1 = d.spo[sp + 1];
    if (g0 == g1) return;
    int a = d.spa[sp], b = d.spb[sp];
    for (int mu = 0; mu < NA; ++mu)
        for (int nu = 0; nu < NB; ++nu) {
            double acc = 0.0;
            for (int g = g0; g < g1; ++g) acc += d.fprim[(size_t)(g - d.cls_off) * NC + mu * NB + nu];
            long long r = d.bfo[a] + mu, c = d.bfo[b] + nu;
            d.F[r * d.nbf + c] += acc;
            if (a != b) d.F[c * d.nbf + r] += acc;
        }
}

// ----------------------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------------------
template <typename T> static const T *boys_tab(pcm_ctx *ctx);
template <> const double *boys_tab<double>(pcm_ctx *ctx) { return ctx->boys64.p; }
template <> const float *boys_tab<float>(pcm_ctx *ctx) { return ctx->boys32.p; }
template <typename T> static const PtInt<T> *points(pcm_mol *mol) {
    return reinterpret_cast<const PtInt<T> *>(sizeof(T) == 8 ? mol->pti64.p : mol->pti32.p);
}

int autotune_pick(pcm_ctx *ctx, const std::string &key, const std::vector<int> &cands,
                  const std::function<void(int)> &launch, int reps) {
    auto f = ctx->tuned.find(key);
    if (f != ctx->tuned.end()) return f->second;
    int best = cands.front();
    if (cands.size() > 1) {
        hipEvent_t a, b;
        HIP_OK(hipEventCreate(&a));
        HIP_OK(hipEventCreate(&b));
        float best_ms = 1e30f;
        for (int c : cands) {
            launch(c);  // warm-up
            float ms_c = 1e30f;
            for (int r = 0; r < reps; ++r) {
                HIP_OK(hipEventRecord(a, ctx->stream));
                launch(c);
                HIP_OK(hipEventRecord(b, ctx->stream));
                HIP_OK(hipEventSynchronize(b));
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, a, b));
                ms_c = std::min(ms_c, ms);
            }
            if (ms_c < best_ms * 0.97f) {  // prefer the earlier (default-like) shape on near ties
                best_ms = ms_c;
                best = c;
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    ctx->tuned[key] = best;
    return best;
}

// Chunk shapes: a (molecule, class) is split into about `target` items (point tiles x pair
// chunks for esp, pair tiles x point chunks for Fock).
constexpr int TARGET_DEFAULT = 4096;
static const std::vector<int> TARGETS{4096, 1024, 2048, 8192, 16384, 32768};

static int esp_chunk_len(long long n_pairs, int M, int target) {
    int tiles = M > 0 ? div_up(M, 256) : 1;
    long long want = (target + tiles - 1) / tiles;
    if (want < 1) want = 1;
    long long len = (n_pairs + want - 1) / want;
    if (len < 16) len = 16;
    return (int)((len + REC_PAD - 1) / REC_PAD * REC_PAD);
}

static int fock_chunk_len(long long n_pairs, int Mpad, int target) {
    int tiles = n_pairs > 0 ? div_up(n_pairs, 256) : 1;
    long long want = (target + tiles - 1) / tiles;
    if (want < 1) want = 1;
    long long len = (Mpad + want - 1) / want;
    if (len < 32) len = 32;
    return (int)((len + PT_BATCH - 1) / PT_BATCH * PT_BATCH);
}

static int ilog2(long long x) {
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

static std::string shape_key(const char *kind, int L, const char *prec, long long n, long long M) {
    return std::string(kind) + ":L" + std::to_string(L) + ":" + prec + ":" + std::to_string(ilog2(n)) + ":" +
           std::to_string(ilog2(M));
}

// Grid of the integral item loops: one item per workgroup and the hardware scheduler balances
// them (items differ in cost: chunk tails, near-field fractions).  Re-staging the Boys table
// per workgroup costs well under 1% of these launches.  The item loop still allows a smaller
// grid (at most 2^30 workgroups).

// device scratch for descriptor tables of one call (all classes uploaded at once)

template <typename T, typename B>
static void esp_class_launch(pcm_ctx *ctx, int L, const EspDesc *d, int nd, long long n_items,
                             hipStream_t stream = nullptr) {
    const B *tab = boys_tab<B>(ctx);
    if (!stream) stream = ctx->stream;
    switch (L) {
#define ESP_CASE(LL)                                                                        \
    case LL:                                                                                \
        k_esp<LL, T, B><<<int_grid(n_items), 256, 0, stream>>>(d, nd, n_items, tab);           \
        break;
        ESP_CASE(0) ESP_CASE(1) ESP_CASE(2) ESP_CASE(3) ESP_CASE(4)
#undef ESP_CASE
    }
    HIP_LAUNCH_OK();
}

template <typename T> static EspDesc esp_desc(pcm_mol *mol, ListSel ls, int cl, int chunk, int row0) {
    PairList &pl = mol->*ls;
    const long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
    const int L = CLS_LA[cl] + CLS_LB[cl];
    EspDesc d{};
    d.rec = pl.rec.p + pl.rec_off[cl];
    d.pts = points<T>(mol);
    d.pperm = mol->pperm.p;
    d.part = mol->part.p;
    d.M = mol->M;
    d.stride = (int)rec_stride<T>(L);
    d.n_pad = (int)((n + REC_PAD - 1) / REC_PAD * REC_PAD);
    d.chunk = chunk;
    d.ntile = div_up(mol->M, 256);
    d.row0 = row0;
    return d;
}

// chunk of (molecule, class), autotuned on first use of its shape key
template <typename T, typename B> static int esp_chunk(pcm_ctx *ctx, pcm_mol *mol, ListSel ls, int cl) {
    const long long n = (mol->*ls).cls_off[cl + 1] - (mol->*ls).cls_off[cl];
    const int L = CLS_LA[cl] + CLS_LB[cl];
    if (!ctx->prm.autotune) return esp_chunk_len(n, mol->M, TARGET_DEFAULT);
    std::vector<int> cands;
    for (int t : TARGETS) {
        int c = esp_chunk_len(n, mol->M, t);
        if (std::find(cands.begin(), cands.end(), c) == cands.end()) cands.push_back(c);
    }
    const std::string key = shape_key("esp", L, prec_tag<T, B>(), n, mol->M);
    if (ctx->tuned.count(key)) {  // cached target for this shape bucket: map it to this size
        return esp_chunk_len(n, mol->M, ctx->tuned[key]);
    }
    int rows_max = 0;
    for (int c : cands) rows_max = std::max(rows_max, div_up(n, c));
    mol->part.ensure((size_t)rows_max * mol->M);
    int best_chunk = autotune_pick(ctx, key + ":chunk", cands, [&](int c) {
        EspDesc d = esp_desc<T>(mol, ls, cl, c, 0);
        d.base = 0;
        long long items = (long long)d.ntile * div_up(n, c);
        EspDesc *dd = (EspDesc *)upload_desc(ctx, &d, sizeof(d));
        esp_class_launch<T, B>(ctx, L, dd, 1, items);
    });
    int target = TARGET_DEFAULT;
    for (int t : TARGETS)
        if (esp_chunk_len(n, mol->M, t) == best_chunk) {
            target = t;
            break;
        }
    ctx->tuned[key] = target;
    return best_chunk;
}

// c[i] = (acc ? c[i] : 0) + the contribution of list `ls` of every molecule
// the descriptor tables of a pass go to `desc` (the context's buffer for an immediate run, a
// buffer of their own for a captured graph)
static unsigned char *upload_tables(pcm_ctx *ctx, DevBuf<unsigned char> &desc, const std::vector<unsigned char> &blob) {
    desc.ensure(std::max<size_t>(blob.size(), size_t(1) << 16));
    if (!blob.empty())
        HIP_OK(hipMemcpyAsync(desc.p, blob.data(), blob.size(), hipMemcpyHostToDevice, ctx->stream));
    return desc.p;
}

template <typename T, typename B>
static void esp_batch_plan(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<double *> &c,
                           ListSel ls, bool acc, DevBuf<unsigned char> &desc, Launches &out) {
    const int n = (int)mols.size();
    std::vector<std::array<int, NCLS>> chunk(n);
    std::vector<int> rows(n, 0);
    for (int i = 0; i < n; ++i) {
        for (int cl = 0; cl < NCLS; ++cl) {
            long long np = (mols[i]->*ls).cls_off[cl + 1] - (mols[i]->*ls).cls_off[cl];
            chunk[i][cl] = np ? esp_chunk<T, B>(ctx, mols[i], ls, cl) : REC_PAD;
            rows[i] += np ? div_up(np, chunk[i][cl]) : 0;
        }
        mols[i]->part.ensure((size_t)std::max(rows[i], 1) * mols[i]->M);
    }
    // descriptors of every class, then the row-sum descriptors
    std::vector<EspDesc> all;
    long long cls_items[NCLS];
    int cls_first[NCLS], cls_n[NCLS];
    std::vector<int> row0(n, 0);
    for (int cl = 0; cl < NCLS; ++cl) {
        cls_first[cl] = (int)all.size();
        long long base = 0;
        for (int i = 0; i < n; ++i) {
            long long np = (mols[i]->*ls).cls_off[cl + 1] - (mols[i]->*ls).cls_off[cl];
            if (!np) continue;
            EspDesc d = esp_desc<T>(mols[i], ls, cl, chunk[i][cl], row0[i]);
            d.base = base;
            base += (long long)d.ntile * div_up(np, chunk[i][cl]);
            row0[i] += div_up(np, chunk[i][cl]);
            all.push_back(d);
        }
        cls_n[cl] = (int)all.size() - cls_first[cl];
        cls_items[cl] = base;
    }
    std::vector<SumDesc> sums;
    long long sbase = 0;
    for (int i = 0; i < n; ++i) {
        SumDesc d{mols[i]->part.p, c[i], sbase, mols[i]->M, rows[i], acc ? 1 : 0};
        sbase += div_up(mols[i]->M, 256);
        sums.push_back(d);
    }
    const size_t eb = all.size() * sizeof(EspDesc), sb = sums.size() * sizeof(SumDesc);
    std::vector<unsigned char> blob(eb + sb);
    if (eb) std::memcpy(blob.data(), all.data(), eb);
    std::memcpy(blob.data() + eb, sums.data(), sb);
    unsigned char *dev = upload_tables(ctx, desc, blob);
    const EspDesc *dd = reinterpret_cast<const EspDesc *>(dev);
    for (int cl = 0; cl < NCLS; ++cl) {
        if (!cls_n[cl]) continue;
        const int L = CLS_LA[cl] + CLS_LB[cl];
        double work = 0.0;
        for (int i = 0; i < n; ++i)
            work += (double)((mols[i]->*ls).cls_off[cl + 1] - (mols[i]->*ls).cls_off[cl]) * mols[i]->M;
        const EspDesc *d0 = dd + cls_first[cl];
        const int nd = cls_n[cl];
        const long long items = cls_items[cl];
        out.add("esp_L" + std::to_string(L) + "_" + prec_tag<T, B>(), work,
                [=](hipStream_t st) { esp_class_launch<T, B>(ctx, L, d0, nd, items, st); });
    }
    const SumDesc *sd = reinterpret_cast<const SumDesc *>(dev + eb);
    out.add("", 0.0, [=](hipStream_t st) {
        k_sum_rows<<<int_grid(sbase), 256, 0, st>>>(sd, n, sbase);
        HIP_LAUNCH_OK();
    });
}

template <typename T, typename B>
static void esp_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<double *> &c, ListSel ls,
                      bool acc) {
    Launches run;
    esp_batch_plan<T, B>(ctx, mols, c, ls, acc, ctx->desc, run);
    run.run(ctx, ctx->stream, ctx->prof);
}

// the launches of run_esp_batch, each pass with a descriptor buffer from `bufs`
void esp_batch_launches(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<double *> &c, int prec,
                        std::vector<std::unique_ptr<DevBuf<unsigned char>>> &bufs, Launches &out) {
    auto buf = [&]() -> DevBuf<unsigned char> & {
        bufs.emplace_back(new DevBuf<unsigned char>());
        return *bufs.back();
    };
    if (prec == PCM_MIXED) {
        esp_batch_plan<double, float>(ctx, mols, c, &pcm_mol::esp, false, buf(), out);
    } else if (prec == PCM_DYNAMIC) {
        esp_batch_plan<double, double>(ctx, mols, c, &pcm_mol::esp, false, buf(), out);
        esp_batch_plan<float, float>(ctx, mols, c, &pcm_mol::esp_w, true, buf(), out);
    } else {
        esp_batch_plan<double, double>(ctx, mols, c, &pcm_mol::esp, false, buf(), out);
    }
}

void run_esp_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<double *> &c, int prec) {
    if (prec == PCM_MIXED) {
        esp_batch<double, float>(ctx, mols, c, &pcm_mol::esp, false);
    } else if (prec == PCM_DYNAMIC) {  // strong pairs in FP64, then the weak ones in FP32 added on
        esp_batch<double, double>(ctx, mols, c, &pcm_mol::esp, false);
        esp_batch<float, float>(ctx, mols, c, &pcm_mol::esp_w, true);
    } else {
        esp_batch<double, double>(ctx, mols, c, &pcm_mol::esp, false);
    }
}

void run_esp(pcm_ctx *ctx, pcm_mol *mol, double *c, int prec) { run_esp_batch(ctx, {mol}, {c}, prec); }

// ---------------------------------------------------------------------------------- Fock
template <typename T, typename B>
static void fock_class_launch(pcm_ctx *ctx, int L, const FockDesc *d, int nd, long long n_items,
                              hipStream_t stream = nullptr) {
    const B *tab = boys_tab<B>(ctx);
    if (!stream) stream = ctx->stream;
    switch (L) {
#define FV_CASE(LL)                                                                                      \
    case LL:                                                                                             \
        k_fock_v<LL, T, B><<<int_grid(n_items), 256, 0, stream>>>(d, nd, n_items, tab);                     \
        break;
        FV_CASE(0) FV_CASE(1) FV_CASE(2) FV_CASE(3) FV_CASE(4)
#undef FV_CASE
    }
    HIP_LAUNCH_OK();
}

template <typename T> static FockDesc fock_desc(pcm_mol *mol, ListSel ls, int cl, int chunk) {
    PairList &pl = mol->*ls;
    FockDesc d{};
    d.rec = pl.rec.p + pl.rec_off[cl];
    d.perm = pair_order(pl, cl);
    d.pts = points<T>(mol);
    d.q = mol->qpad.p;
    d.vout = mol->vbuf.p;
    d.n_pairs = (int)(pl.cls_off[cl + 1] - pl.cls_off[cl]);
    d.Mpad = mol->Mpad;
    d.chunk = chunk;
    d.nptile = div_up(d.n_pairs, 256);
    d.stride = (int)align16(sizeof(PairHdr<T>));
    return d;
}

template <typename T, typename B> static int fock_chunk(pcm_ctx *ctx, pcm_mol *mol, ListSel ls, int cl) {
    const long long n = (mol->*ls).cls_off[cl + 1] - (mol->*ls).cls_off[cl];
    const int L = CLS_LA[cl] + CLS_LB[cl];
    if (!ctx->prm.autotune) return fock_chunk_len(n, mol->Mpad, TARGET_DEFAULT);
    const std::string key = shape_key("fock", L, prec_tag<T, B>(), n, mol->M);
    if (ctx->tuned.count(key)) return fock_chunk_len(n, mol->Mpad, ctx->tuned[key]);
    std::vector<int> cands;
    for (int t : TARGETS) {
        int c = fock_chunk_len(n, mol->Mpad, t);
        if (std::find(cands.begin(), cands.end(), c) == cands.end()) cands.push_back(c);
    }
    int best_chunk = autotune_pick(ctx, key + ":chunk", cands, [&](int c) {
        FockDesc d = fock_desc<T>(mol, ls, cl, c);
        d.base = 0;
        long long items = (long long)d.nptile * div_up(mol->Mpad, c);
        FockDesc *dd = (FockDesc *)upload_desc(ctx, &d, sizeof(d));
        fock_class_launch<T, B>(ctx, L, dd, 1, items);
    });
    int target = TARGET_DEFAULT;
    for (int t : TARGETS)
        if (fock_chunk_len(n, mol->Mpad, t) == best_chunk) {
            target = t;
            break;
        }
    ctx->tuned[key] = target;
    return best_chunk;
}

// V buffer and primitive-block buffer large enough for every class and every tuning candidate
void fock_buffers(pcm_mol *mol, ListSel ls) {
    PairList &pl = mol->*ls;
    size_t vneed = 0, fneed = 0;
    for (int cl = 0; cl < NCLS; ++cl) {
        long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        int cmin = fock_chunk_len(n, mol->Mpad, TARGET_DEFAULT);
        for (int t : TARGETS) cmin = std::min(cmin, fock_chunk_len(n, mol->Mpad, t));
        size_t v = (size_t)div_up(mol->Mpad, cmin) * ntuv(CLS_LA[cl] + CLS_LB[cl]) * n;
        vneed = std::max(vneed, v);
        fneed = std::max(fneed, (size_t)n * ncart(CLS_LA[cl]) * ncart(CLS_LB[cl]));
    }
    mol->vbuf.ensure(vneed + 1);
    mol->fprim.ensure(fneed + 1);
}

// charges into the padded copy the point loops read (the tail past M stays zero)
__global__ void k_copy_q(const double *__restrict__ q, double *__restrict__ qpad, int M) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) qpad[k] = q[k];
}

template <typename T, typename B>
static void fock_batch_plan(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &q,
                            const std::vector<double *> &F, ListSel ls, DevBuf<unsigned char> &desc,
                            Launches &out) {
    const int n = (int)mols.size();
    for (int i = 0; i < n; ++i) {
        fock_buffers(mols[i], ls);
        const int M = mols[i]->M;
        const double *qi = q[i];
        double *qp = mols[i]->qpad.p;
        out.add("", 0.0, [=](hipStream_t st) {
            k_copy_q<<<grid_for(M, 256), 256, 0, st>>>(qi, qp, M);
            HIP_LAUNCH_OK();
        });
    }
    std::vector<std::array<int, NCLS>> chunk(n);
    for (int i = 0; i < n; ++i)
        for (int cl = 0; cl < NCLS; ++cl)
            chunk[i][cl] = (mols[i]->*ls).cls_off[cl + 1] > (mols[i]->*ls).cls_off[cl]
                               ? fock_chunk<T, B>(ctx, mols[i], ls, cl)
                               : PT_BATCH;
    std::vector<FockDesc> all;
    long long cls_items[NCLS];
    int cls_first[NCLS], cls_n[NCLS];
    for (int cl = 0; cl < NCLS; ++cl) {
        cls_first[cl] = (int)all.size();
        long long base = 0;
        for (int i = 0; i < n; ++i) {
            if ((mols[i]->*ls).cls_off[cl + 1] == (mols[i]->*ls).cls_off[cl]) continue;
            FockDesc d = fock_desc<T>(mols[i], ls, cl, chunk[i][cl]);
            d.base = base;
            base += (long long)d.nptile * div_up(mols[i]->Mpad, chunk[i][cl]);
            all.push_back(d);
        }
        cls_n[cl] = (int)all.size() - cls_first[cl];
        cls_items[cl] = base;
    }
    // contraction / scatter descriptors of every class (one per molecule with pairs in the class)
    std::vector<FockCDesc> cds;
    int c_first[NCLS], c_n[NCLS];
    long long c_items[NCLS], s_items[NCLS];
    for (int cl = 0; cl < NCLS; ++cl) {
        c_first[cl] = (int)cds.size();
        long long base = 0, sbase = 0;
        for (int i = 0; i < n; ++i) {
            pcm_mol *mol = mols[i];
            PairList &pl = mol->*ls;
            const long long np = pl.cls_off[cl + 1] - pl.cls_off[cl];
            if (!np) continue;
            FockCDesc d{};
            d.base = base;
            d.sbase = sbase;
            d.n = np;
            d.sp0 = mol->sp_cls_off[cl];
            d.nsp = mol->sp_cls_off[cl + 1] - d.sp0;
            d.cls_off = pl.cls_off[cl];
            d.nch = div_up(mol->Mpad, chunk[i][cl]);
            d.nbf = mol->nbf;
            d.vnt = ntuv(CLS_LA[cl] + CLS_LB[cl]);
            d.memb = nullptr;
            d.vin = mol->vbuf.p;
            d.vperm = pair_order(pl, cl);
            d.es = pl.ent_sp.p + pl.cls_off[cl];
            d.ei = pl.ent_ij.p + pl.cls_off[cl];
            d.spo = pl.spo.p;
            d.spa = mol->spa.p;
            d.spb = mol->spb.p;
            d.snp = mol->snp.p;
            d.soff = mol->soff.p;
            d.satom = mol->satom.p;
            d.cnoff = mol->cnoff.p;
            d.bfo = mol->bfo.p;
            d.pexp = mol->pexp.p;
            d.cn = mol->cn.p;
            d.xyz = mol->xyz.p;
            d.fprim = mol->fprim.p;
            d.F = F[i];
            base += np;
            sbase += d.nsp;
            cds.push_back(d);
        }
        c_n[cl] = (int)cds.size() - c_first[cl];
        c_items[cl] = base;
        s_items[cl] = sbase;
    }
    const size_t fb = all.size() * sizeof(FockDesc), cb = cds.size() * sizeof(FockCDesc);
    std::vector<unsigned char> blob(fb + cb);
    if (fb) std::memcpy(blob.data(), all.data(), fb);
    if (cb) std::memcpy(blob.data() + fb, cds.data(), cb);
    unsigned char *dev = upload_tables(ctx, desc, blob);
    const FockDesc *dd = reinterpret_cast<const FockDesc *>(dev);
    const FockCDesc *cd = reinterpret_cast<const FockCDesc *>(dev + fb);
    for (int cl = 0; cl < NCLS; ++cl) {
        if (!cls_n[cl]) continue;
        const int L = CLS_LA[cl] + CLS_LB[cl];
        double work = 0.0;
        for (int i = 0; i < n; ++i)
            work += (double)((mols[i]->*ls).cls_off[cl + 1] - (mols[i]->*ls).cls_off[cl]) * mols[i]->M;
        const FockDesc *d0 = dd + cls_first[cl];
        const int nd = cls_n[cl];
        const long long items = cls_items[cl];
        out.add("fock_v_L" + std::to_string(L) + "_" + prec_tag<T, B>(), work,
                [=](hipStream_t st) { fock_class_launch<T, B>(ctx, L, d0, nd, items, st); });
        const FockCDesc *cdc = cd + c_first[cl];
        const int ncd = c_n[cl];
        const long long np = c_items[cl], nsp = s_items[cl];
        const int g = grid_for(np, 128), gs = grid_for(nsp, 128);
        out.add("fock_contract", (double)np, [=](hipStream_t st) {
#define FC_CASE(CI, LA_, LB_)                                                                                      \
    case CI:                                                                                                       \
        k_fock_contract<LA_, LB_><<<g, 128, 0, st>>>(cdc, ncd, np);                                                \
        HIP_LAUNCH_OK();                                                                                           \
        k_fock_scatter<LA_, LB_><<<gs, 128, 0, st>>>(cdc, ncd, nsp);                                               \
        break;
#define FCW_CASE(CI, LA_, LB_)                                                                                     \
    case CI:                                                                                                       \
        k_fock_contract_w<LA_, LB_><<<grid_for(np, FCW_WAVES), 64 * FCW_WAVES, 0, st>>>(cdc, ncd, np);              \
        HIP_LAUNCH_OK();                                                                                           \
        k_fock_scatter<LA_, LB_><<<gs, 128, 0, st>>>(cdc, ncd, nsp);                                               \
        break;
            switch (cl) {
                FC_CASE(0, 0, 0)
                FC_CASE(1, 0, 1)
                FC_CASE(2, 0, 2)
                FC_CASE(3, 1, 1)
                FCW_CASE(4, 1, 2)
                FCW_CASE(5, 2, 2)
            }
#undef FC_CASE
#undef FCW_CASE
            HIP_LAUNCH_OK();
        });
    }
}

template <typename T, typename B>
static void fock_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &q,
                       const std::vector<double *> &F, ListSel ls) {
    Launches run;
    fock_batch_plan<T, B>(ctx, mols, q, F, ls, ctx->desc, run);
    run.run(ctx, ctx->stream, ctx->prof);
}

// the launches of run_fock_batch, each pass with a descriptor buffer from `bufs`
void fock_batch_launches(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &q,
                         const std::vector<double *> &F, int prec,
                         std::vector<std::unique_ptr<DevBuf<unsigned char>>> &bufs, Launches &out) {
    auto buf = [&]() -> DevBuf<unsigned char> & {
        bufs.emplace_back(new DevBuf<unsigned char>());
        return *bufs.back();
    };
    if (prec == PCM_MIXED) {
        fock_batch_plan<double, float>(ctx, mols, q, F, &pcm_mol::fock, buf(), out);
    } else if (prec == PCM_DYNAMIC) {
        fock_batch_plan<double, double>(ctx, mols, q, F, &pcm_mol::fock, buf(), out);
        fock_batch_plan<float, float>(ctx, mols, q, F, &pcm_mol::fock_w, buf(), out);
    } else {
        fock_batch_plan<double, double>(ctx, mols, q, F, &pcm_mol::fock, buf(), out);
    }
}

void run_fock_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &q,
                    const std::vector<double *> &F, int prec) {
    if (prec == PCM_MIXED) {
        fock_batch<double, float>(ctx, mols, q, F, &pcm_mol::fock);
    } else if (prec == PCM_DYNAMIC) {  // both lists add their blocks to F
        fock_batch<double, double>(ctx, mols, q, F, &pcm_mol::fock);
        fock_batch<float, float>(ctx, mols, q, F, &pcm_mol::fock_w);
    } else {
        fock_batch<double, double>(ctx, mols, q, F, &pcm_mol::fock);
    }
}

void run_fock(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F, int prec) {
    run_fock_batch(ctx, {mol}, {q}, {F}, prec);
}

void run_fock_lists(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F, int prec, ListSel strong, ListSel weak) {
    if (prec == PCM_MIXED) {
        fock_batch<double, float>(ctx, {mol}, {q}, {F}, strong);
    } else {
        fock_batch<double, double>(ctx, {mol}, {q}, {F}, strong);
        if (prec == PCM_DYNAMIC) fock_batch<float, float>(ctx, {mol}, {q}, {F}, weak);
    }
}

// Contraction to F blocks and scatter into F (one molecule, class cl of list pl) of V sums that
// another pass accumulated: vin[(c * vnt + t) * n + q] for chunk c < nch, vnt >= ntuv(L); with
// memb, entries of pl whose bit is clear add zero blocks (pl is then a merged list).
void fock_contract_scatter(pcm_ctx *ctx, pcm_mol *mol, const PairList &pl, int cl, const double *vin, int nch,
                           int vnt, const unsigned long long *memb, double *F) {
    const long long np = pl.cls_off[cl + 1] - pl.cls_off[cl];
    const long long nsp = mol->sp_cls_off[cl + 1] - mol->sp_cls_off[cl];
    if (np == 0 || nsp == 0) return;
    FockCDesc d{};
    d.base = 0;
    d.sbase = 0;
    d.n = np;
    d.sp0 = mol->sp_cls_off[cl];
    d.nsp = nsp;
    d.cls_off = pl.cls_off[cl];
    d.nch = nch;
    d.nbf = mol->nbf;
    d.vnt = vnt;
    d.memb = memb;
    d.vin = vin;
    d.vperm = pair_order(pl, cl);
    d.es = pl.ent_sp.p + pl.cls_off[cl];
    d.ei = pl.ent_ij.p + pl.cls_off[cl];
    d.spo = pl.spo.p;
    d.spa = mol->spa.p;
    d.spb = mol->spb.p;
    d.snp = mol->snp.p;
    d.soff = mol->soff.p;
    d.satom = mol->satom.p;
    d.cnoff = mol->cnoff.p;
    d.bfo = mol->bfo.p;
    d.pexp = mol->pexp.p;
    d.cn = mol->cn.p;
    d.xyz = mol->xyz.p;
    d.fprim = mol->fprim.p;
    d.F = F;
    const FockCDesc *cdc = (const FockCDesc *)upload_desc(ctx, &d, sizeof(d));
    const int g = grid_for(np, 128), gs = grid_for(nsp, 128);
    ProfScope ps(ctx, "fock_contract", (double)np);
#define FC_CASE(CI, LA_, LB_)                                                                                      \
    case CI:                                                                                                       \
        k_fock_contract<LA_, LB_><<<g, 128, 0, ctx->stream>>>(cdc, 1, np);                                         \
        HIP_LAUNCH_OK();                                                                                           \
        k_fock_scatter<LA_, LB_><<<gs, 128, 0, ctx->stream>>>(cdc, 1, nsp);                                        \
        break;
#define FCW_CASE(CI, LA_, LB_)                                                                                     \
    case CI:                                                                                                       \
        k_fock_contract_w<LA_, LB_><<<grid_for(np, FCW_WAVES), 64 * FCW_WAVES, 0, ctx->stream>>>(cdc, 1, np);       \
        HIP_LAUNCH_OK();                                                                                           \
        k_fock_scatter<LA_, LB_><<<gs, 128, 0, ctx->stream>>>(cdc, 1, nsp);                                        \
        break;
    switch (cl) {
        FC_CASE(0, 0, 0)
        FC_CASE(1, 0, 1)
        FC_CASE(2, 0, 2)
        FC_CASE(3, 1, 1)
        FCW_CASE(4, 1, 2)
        FCW_CASE(5, 2, 2)
    }
#undef FC_CASE
#undef FCW_CASE
    HIP_LAUNCH_OK();
}
