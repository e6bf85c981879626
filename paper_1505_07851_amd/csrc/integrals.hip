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
#include "pcm_internal.h"

// ----------------------------------------------------------------------------------------
// esp: partial c over one chunk of pairs of one class
// ----------------------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(256) void k_esp(const unsigned char *__restrict__ rec, int stride, int n_pad,
                                             int chunk_len, const PtInt<T> *__restrict__ pts, int M,
                                             const T *__restrict__ boys_g, double *__restrict__ part, int row0) {
    constexpr int NT = ntuv(L), PB = pair_batch<L>();
    __shared__ T tab[BoysCfg<T>::NROW * BoysCfg<T>::MT];
    load_boys<T>(tab, boys_g);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const PtInt<T> me = pts[k < M ? k : M - 1];
    const int p0 = blockIdx.y * chunk_len;
    const int p1 = min(n_pad, p0 + chunk_len);
    double acc = 0.0;
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
            T R[NT];
            eval_R<L, T>(h[b].Px - me.x, h[b].Py - me.y, h[b].Pz - me.z, h[b], me.zeta2, me.zeta, me.lim, tab, R);
            T s = T(0);
#pragma unroll
            for (int t = 0; t < NT; ++t) s = fma(D[b][t], R[t], s);
            acc += (double)s;
        }
    }
    if (k < M) part[(size_t)(row0 + blockIdx.y) * M + k] = acc;
}

// fixed-order sum of partial rows: out[k] = sum_r part[r*M + k]
__global__ void k_sum_rows(const double *__restrict__ part, int rows, int M, double *__restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += part[(size_t)r * M + k];
    out[k] = s;
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

void run_bz(pcm_ctx *ctx, pcm_mol *mol, double *bz) {
    ProfScope ps(ctx, "bz", (double)mol->M * mol->N);
    k_bz<<<div_up(mol->M, 256), 256, 0, ctx->stream>>>(mol->px.p, mol->py.p, mol->pz.p, mol->M, mol->zeta.p,
                                                          mol->xyz.p, mol->Z.p, mol->N, bz);
    HIP_LAUNCH_OK();
}

// ----------------------------------------------------------------------------------------
// launch geometry
// ----------------------------------------------------------------------------------------
static int target_groups() { return 4096; }

static int esp_chunk_len(long long n_pairs, int M) {
    int tiles = M > 0 ? div_up(M, 256) : 1;
    long long want = (target_groups() + tiles - 1) / tiles;
    if (want < 1) want = 1;
    long long len = (n_pairs + want - 1) / want;
    if (len < 16) len = 16;
    return (int)((len + REC_PAD - 1) / REC_PAD * REC_PAD);
}

template <typename T> static const T *boys_tab(pcm_ctx *ctx);
template <> const double *boys_tab<double>(pcm_ctx *ctx) { return ctx->boys64.p; }
template <> const float *boys_tab<float>(pcm_ctx *ctx) { return ctx->boys32.p; }
template <typename T> static const PtInt<T> *points(pcm_mol *mol) {
    return reinterpret_cast<const PtInt<T> *>(sizeof(T) == 8 ? mol->pti64.p : mol->pti32.p);
}

template <typename T>
static void esp_launch(pcm_ctx *ctx, pcm_mol *mol, double *c) {
    PairList &pl = mol->esp;
    const int M = mol->M;
    int rows = 0;
    int chunk[NCLS];
    for (int cl = 0; cl < NCLS; ++cl) {
        long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        chunk[cl] = n ? esp_chunk_len(n, M) : REC_PAD;
        rows += n ? div_up(n, chunk[cl]) : 0;
    }
    if (rows == 0) {
        HIP_OK(hipMemsetAsync(c, 0, sizeof(double) * M, ctx->stream));
        return;
    }
    mol->part.ensure((size_t)rows * M);
    const T *tab = boys_tab<T>(ctx);
    int row0 = 0;
    for (int cl = 0; cl < NCLS; ++cl) {
        long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        if (!n) continue;
        int L = CLS_LA[cl] + CLS_LB[cl];
        int n_pad = (int)((n + REC_PAD - 1) / REC_PAD * REC_PAD);
        int nch = div_up(n, chunk[cl]);
        dim3 grid(div_up(M, 256), nch);
        const unsigned char *rec = pl.rec.p + pl.rec_off[cl];
        int stride = (int)rec_stride<T>(L);
        {
            ProfScope ps(ctx, "esp_L" + std::to_string(L) + (sizeof(T) == 8 ? "_f64" : "_f32"), (double)n * M);
            switch (L) {
#define ESP_CASE(LL)                                                                                                  \
    case LL:                                                                                                          \
        k_esp<LL, T><<<grid, 256, 0, ctx->stream>>>(rec, stride, n_pad, chunk[cl], points<T>(mol), M, tab, mol->part.p, \
                                                    row0);                                                             \
        break;
                ESP_CASE(0) ESP_CASE(1) ESP_CASE(2) ESP_CASE(3) ESP_CASE(4)
#undef ESP_CASE
            }
            HIP_LAUNCH_OK();
        }
        row0 += nch;
    }
    k_sum_rows<<<div_up(M, 256), 256, 0, ctx->stream>>>(mol->part.p, rows, M, c);
    HIP_LAUNCH_OK();
}

void run_esp(pcm_ctx *ctx, pcm_mol *mol, double *c, int prec) {
    if (prec == PCM_MIXED)
        esp_launch<float>(ctx, mol, c);
    else
        esp_launch<double>(ctx, mol, c);
}

// ----------------------------------------------------------------------------------------
// Fock: V_tuv(pair) = sum_k q_k R_tuv(pair, k) over one chunk of points
// ----------------------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(256) void k_fock_v(const unsigned char *__restrict__ rec, int stride, int n_pairs,
                                                const PtInt<T> *__restrict__ pts, const double *__restrict__ q,
                                                int Mpad, int chunk_len, const T *__restrict__ boys_g,
                                                double *__restrict__ vout) {
    constexpr int NT = ntuv(L);
    __shared__ T tab[BoysCfg<T>::NROW * BoysCfg<T>::MT];
    load_boys<T>(tab, boys_g);
    const int ip = blockIdx.x * blockDim.x + threadIdx.x;
    const PairHdr<T> h = *reinterpret_cast<const PairHdr<T> *>(rec + (size_t)(ip < n_pairs ? ip : n_pairs - 1) * stride);
    const int k0 = blockIdx.y * chunk_len;
    const int k1 = min(Mpad, k0 + chunk_len);
    double V[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) V[t] = 0.0;
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
            T R[NT];
            eval_R<L, T>(h.Px - pt[b].x, h.Py - pt[b].y, h.Pz - pt[b].z, h, pt[b].zeta2, pt[b].zeta, pt[b].lim, tab,
                         R);
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

// per primitive pair: F_prim[mu nu] = -c_mu_i c_nu_j sum_tuv E^{mu nu}_tuv V_tuv
template <int LA, int LB>
__global__ void k_fock_contract(long long n, int nch, const double *__restrict__ vin, const int *__restrict__ ent_sp,
                                const int *__restrict__ ent_ij, const int *__restrict__ spa,
                                const int *__restrict__ spb, const int *__restrict__ snp, const int *__restrict__ soff,
                                const int *__restrict__ satom, const int *__restrict__ cnoff,
                                const double *__restrict__ pexp, const double *__restrict__ cn,
                                const double *__restrict__ xyz, double *__restrict__ fprim) {
    constexpr int L = LA + LB, NT = ntuv(L), NC = ncart(LA) * ncart(LB);
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
    double P[3] = {(ea * A[0] + eb * B[0]) / p, (ea * A[1] + eb * B[1]) / p, (ea * A[2] + eb * B[2]) / p};
    Herm1D<LA, LB> ex, ey, ez;
    double inv2p = 0.5 / p;
    ex.build(P[0] - A[0], P[0] - B[0], inv2p);
    ey.build(P[1] - A[1], P[1] - B[1], inv2p);
    ez.build(P[2] - A[2], P[2] - B[2], inv2p);
    for (int mu = 0; mu < ncart(LA); ++mu) {
        int ax, ay, az;
        cart_comp(LA, mu, ax, ay, az);
        double cmu = cn[cnoff[a] + mu * snp[a] + i];
        for (int nu = 0; nu < ncart(LB); ++nu) {
            int bx, by, bz;
            cart_comp(LB, nu, bx, by, bz);
            double s = 0.0;
            for (int t = 0; t <= ax + bx; ++t)
                for (int u = 0; u <= ay + by; ++u) {
                    double etu = ex.e[ax][bx][t] * ey.e[ay][by][u];
                    for (int v = 0; v <= az + bz; ++v) s += etu * ez.e[az][bz][v] * V[tuv_idx(t, u, v)];
                }
            fprim[(size_t)q * NC + mu * ncart(LB) + nu] = -cmu * cn[cnoff[b] + nu * snp[b] + j] * s;
        }
    }
}

// per candidate shell pair: sum its primitive pairs in list order and add the block to F
template <int LA, int LB>
__global__ void k_fock_scatter(long long sp0, long long nsp, long long cls_off, const int *__restrict__ spo,
                               const int *__restrict__ spa, const int *__restrict__ spb, const int *__restrict__ bfo,
                               const double *__restrict__ fprim, int nbf, double *__restrict__ F) {
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = NA * NB;
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsp) return;
    long long sp = sp0 + s;
    int g0 = spo[sp], g1 = spo[sp + 1];
    if (g0 == g1) return;
    int a = spa[sp], b = spb[sp];
    for (int mu = 0; mu < NA; ++mu)
        for (int nu = 0; nu < NB; ++nu) {
            double acc = 0.0;
            for (int g = g0; g < g1; ++g) acc += fprim[(size_t)(g - cls_off) * NC + mu * NB + nu];
            long long r = bfo[a] + mu, c = bfo[b] + nu;
            F[r * nbf + c] += acc;
            if (a != b) F[c * nbf + r] += acc;
        }
}

static int fock_chunk_len(long long n_pairs, int Mpad) {
    int tiles = n_pairs > 0 ? div_up(n_pairs, 256) : 1;
    long long want = (target_groups() + tiles - 1) / tiles;
    if (want < 1) want = 1;
    long long len = (Mpad + want - 1) / want;
    if (len < 32) len = 32;
    return (int)((len + PT_BATCH - 1) / PT_BATCH * PT_BATCH);
}

template <typename T>
static void fock_launch(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F) {
    PairList &pl = mol->fock;
    const int M = mol->M, Mpad = mol->Mpad;
    const T *tab = boys_tab<T>(ctx);
    HIP_OK(hipMemcpyAsync(mol->qpad.p, q, sizeof(double) * M, hipMemcpyDeviceToDevice, ctx->stream));
    size_t vneed = 0, fneed = 0;
    int chunk[NCLS];
    for (int cl = 0; cl < NCLS; ++cl) {
        long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        chunk[cl] = fock_chunk_len(n, Mpad);
        int nch = div_up(Mpad, chunk[cl]);
        size_t v = (size_t)nch * ntuv(CLS_LA[cl] + CLS_LB[cl]) * n;
        vneed = v > vneed ? v : vneed;
        size_t f = (size_t)n * ncart(CLS_LA[cl]) * ncart(CLS_LB[cl]);
        fneed = f > fneed ? f : fneed;
    }
    mol->vbuf.ensure(vneed + 1);
    mol->fprim.ensure(fneed + 1);
    for (int cl = 0; cl < NCLS; ++cl) {
        long long n = pl.cls_off[cl + 1] - pl.cls_off[cl];
        if (!n) continue;
        int L = CLS_LA[cl] + CLS_LB[cl];
        int nch = div_up(Mpad, chunk[cl]);
        dim3 grid(div_up(n, 256), nch);
        const unsigned char *rec = pl.rec.p + pl.rec_off[cl];
        int stride = (int)align16(sizeof(PairHdr<T>));
        {
            ProfScope ps(ctx, "fock_v_L" + std::to_string(L) + (sizeof(T) == 8 ? "_f64" : "_f32"), (double)n * M);
            switch (L) {
#define FV_CASE(LL)                                                                                                 \
    case LL:                                                                                                        \
        k_fock_v<LL, T><<<grid, 256, 0, ctx->stream>>>(rec, stride, (int)n, points<T>(mol), mol->qpad.p, Mpad,      \
                                                       chunk[cl], tab, mol->vbuf.p);                                \
        break;
                FV_CASE(0) FV_CASE(1) FV_CASE(2) FV_CASE(3) FV_CASE(4)
#undef FV_CASE
            }
            HIP_LAUNCH_OK();
        }
        const int *es = pl.ent_sp.p + pl.cls_off[cl], *ei = pl.ent_ij.p + pl.cls_off[cl];
        long long sp0 = mol->sp_cls_off[cl], nsp = mol->sp_cls_off[cl + 1] - sp0;
        int g = div_up(n, 128), gs = div_up(nsp, 128);
        ProfScope ps2(ctx, "fock_contract", (double)n);
#define FC_CASE(CI, LA_, LB_)                                                                                      \
    case CI:                                                                                                       \
        k_fock_contract<LA_, LB_><<<g, 128, 0, ctx->stream>>>(n, nch, mol->vbuf.p, es, ei, mol->spa.p, mol->spb.p, \
                                                              mol->snp.p, mol->soff.p, mol->satom.p, mol->cnoff.p, \
                                                              mol->pexp.p, mol->cn.p, mol->xyz.p, mol->fprim.p);   \
        HIP_LAUNCH_OK();                                                                                           \
        k_fock_scatter<LA_, LB_><<<gs, 128, 0, ctx->stream>>>(sp0, nsp, pl.cls_off[cl], pl.spo.p, mol->spa.p,      \
                                                              mol->spb.p, mol->bfo.p, mol->fprim.p, mol->nbf, F);  \
        break;
        switch (cl) {
            FC_CASE(0, 0, 0)
            FC_CASE(1, 0, 1)
            FC_CASE(2, 0, 2)
            FC_CASE(3, 1, 1)
            FC_CASE(4, 1, 2)
            FC_CASE(5, 2, 2)
        }
#undef FC_CASE
        HIP_LAUNCH_OK();
    }
}

void run_fock(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F, int prec) {
    if (prec == PCM_MIXED)
        fock_launch<float>(ctx, mol, q, F);
    else
        fock_launch<double>(ctx, mol, q, F);
}
