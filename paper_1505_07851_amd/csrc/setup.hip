// Setup kernels: Boys tables, device prefix sums, the ISWIG surface (Sec. 2, Eqs. 3, 7, 9;
// Sec. 3), basis normalisation (Eqs. 11-12), screened primitive-pair lists (Sec. 4a,
// Eqs. 15, 18) and the per-pair records consumed by the integral kernels.
//
// This translation unit is compiled without floating-point contraction so that the
// keep/screen decisions evaluate the same IEEE expressions as a plain C reading of the
// formulas.
#include "pcm_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstring>

// ----------------------------------------------------------------------------------------
// Boys tables (host generation, once per context)
// ----------------------------------------------------------------------------------------
static void boys_host(int mmax, long double T, long double *F) {
    long double term = 1.0L / (2 * mmax + 1), sum = term;
    for (int i = 1; i < 4000; ++i) {
        term *= 2.0L * T / (long double)(2 * mmax + 2 * i + 1);
        sum += term;
        if (term < 1e-22L * sum) break;
    }
    long double e = expl(-T);
    F[mmax] = e * sum;
    for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0L * T * F[m + 1] + e) / (2 * m + 1);
}

void ctx_ensure_device(pcm_ctx *ctx) {
    if (ctx->dev_ready) return;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    ctx->device = dev;
    using C64 = BoysCfg<double>;
    using C32 = BoysCfg<float>;
    std::vector<double> t64(C64::NROW * C64::MT);
    std::vector<float> t32(C32::NROW * C32::MT);
    long double F[32];
    for (int i = 0; i < C64::NROW; ++i) {
        boys_host(C64::MT - 1, (long double)i / 8.0L, F);
        for (int m = 0; m < C64::MT; ++m) t64[i * C64::MT + m] = (double)F[m];
    }
    for (int i = 0; i < C32::NROW; ++i) {
        boys_host(C32::MT - 1, (long double)i / 8.0L, F);
        for (int m = 0; m < C32::MT; ++m) t32[i * C32::MT + m] = (float)F[m];
    }
    ctx->boys64.ensure(t64.size());
    ctx->boys32.ensure(t32.size());
    ctx->scal.ensure(4096);
    ctx->iscal.ensure(64);
    ctx->lscal.ensure(64);
    HIP_OK(hipMemcpyAsync(ctx->boys64.p, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(ctx->boys32.p, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    noalloc_scratch_init(dev);
    ctx->dev_ready = true;
}

// ----------------------------------------------------------------------------------------
// exclusive prefix sum of int32 (deterministic, two-level recursive)
// ----------------------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_B = SCAN_T * SCAN_I;

__global__ __launch_bounds__(SCAN_T) void k_scan_block(const int *__restrict__ in, int *__restrict__ out,
                                                        int *__restrict__ bsum, long long n) {
    __shared__ int s[SCAN_T];
    const int tid = threadIdx.x;
    const long long base = (long long)blockIdx.x * SCAN_B + (long long)tid * SCAN_I;
    int v[SCAN_I];
    int tsum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        long long idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        tsum += v[i];
    }
    s[tid] = tsum;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int t = tid >= off ? s[tid - off] : 0;
        __syncthreads();
        s[tid] += t;
        __syncthreads();
    }
    int run = s[tid] - tsum;
    if (tid == SCAN_T - 1) bsum[blockIdx.x] = s[tid];
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        long long idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
}

__global__ void k_scan_add(int *__restrict__ out, const int *__restrict__ boff, long long n) {
    long long idx = (long long)blockIdx.x * SCAN_B + threadIdx.x;
    int add = boff[blockIdx.x];
    for (int i = 0; i < SCAN_I; ++i, idx += SCAN_T)
        if (idx < n) out[idx] += add;
}

static void scan_rec(pcm_ctx *ctx, const int *in, int *out, long long n, int *tmp, int *total_dev) {
    long long nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb <= 1) {
        k_scan_block<<<1, SCAN_T, 0, ctx->stream>>>(in, out, total_dev, n);
        HIP_LAUNCH_OK();
        return;
    }
    int *bsum = tmp, *boff = tmp + nb;
    k_scan_block<<<(unsigned)nb, SCAN_T, 0, ctx->stream>>>(in, out, bsum, n);
    HIP_LAUNCH_OK();
    scan_rec(ctx, bsum, boff, nb, tmp + 2 * nb, total_dev);
    k_scan_add<<<(unsigned)nb, SCAN_T, 0, ctx->stream>>>(out, boff, n);
    HIP_LAUNCH_OK();
}

// exclusive prefix sum on the stream; returns the device address of the total (n >= 1)
static int *scan_exclusive_dev(pcm_ctx *ctx, pcm_mol *mol, const int *in, int *out, long long n) {
    long long need = 16, m = n;
    while (m > 1) {
        m = (m + SCAN_B - 1) / SCAN_B;
        need += 2 * m + 2;
    }
    mol->scan_tmp.ensure(need + 1);
    int *tot = mol->scan_tmp.p + need;
    scan_rec(ctx, in, out, n, mol->scan_tmp.p, tot);
    return tot;
}

void scan_exclusive(pcm_ctx *ctx, pcm_mol *mol, const int *in, int *out, long long n, long long *total) {
    if (n <= 0) {
        if (total) *total = 0;
        return;
    }
    int *tot = scan_exclusive_dev(ctx, mol, in, out, n);
    if (total) {
        int t = 0;
        HIP_OK(hipMemcpyAsync(&t, tot, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        *total = t;
    }
}

// ----------------------------------------------------------------------------------------
// ISWIG surface (Sec. 2, Eqs. 3, 7, 9).  Point (I, j): r = R_I + rho_I u_j,
// zeta = zeta0 / (rho_I sqrt(w_j)), S = prod_{J != I} S_wf with
// S_wf = 1/2 [erfc(zeta (R_J - d)) + erfc(zeta (R_J + d))] (the cancellation-free form of
// Eq. 9); atoms with zeta (d - R_J) >= 6 give S_wf = 1 to double precision and are skipped.
// ----------------------------------------------------------------------------------------
__device__ double switching_product(const double *__restrict__ xyz, const double *__restrict__ rad, int N, int I,
                                    double x, double y, double z, double zeta) {
    double s = 1.0;
    const double reach = 6.0 / zeta;
    for (int J = 0; J < N; ++J) {
        if (J == I) continue;
        double dx = x - xyz[3 * J], dy = y - xyz[3 * J + 1], dz = z - xyz[3 * J + 2];
        double d = sqrt(dx * dx + dy * dy + dz * dz);
        if (d >= rad[J] + reach) continue;
        s *= 0.5 * (erfc(zeta * (rad[J] - d)) + erfc(zeta * (rad[J] + d)));
    }
    return s;
}

// raw pass: keep flag per raw point
__global__ void k_surface_flags(const double *__restrict__ xyz, const double *__restrict__ rad, int N,
                                const double *__restrict__ dirs, const double *__restrict__ w, int nsph,
                                double zeta0, double thresh, int *__restrict__ flag) {
    int kr = blockIdx.x * blockDim.x + threadIdx.x;
    if (kr >= N * nsph) return;
    int I = kr / nsph, j = kr - I * nsph;
    double zeta = zeta0 / (rad[I] * sqrt(w[j]));
    double x = xyz[3 * I] + rad[I] * dirs[3 * j];
    double y = xyz[3 * I + 1] + rad[I] * dirs[3 * j + 1];
    double z = xyz[3 * I + 2] + rad[I] * dirs[3 * j + 2];
    double s = switching_product(xyz, rad, N, I, x, y, z, zeta);
    flag[kr] = s >= thresh ? 1 : 0;
}

__global__ void k_surface_compact(const int *__restrict__ flag, const int *__restrict__ pos, int nraw,
                                  int *__restrict__ keep) {
    int kr = blockIdx.x * blockDim.x + threadIdx.x;
    if (kr >= nraw) return;
    if (flag[kr]) keep[pos[kr]] = kr;
}

// kept pass: positions (from atoms, or explicit), S, A_kk and packed point records
__global__ void k_surface_points(const double *__restrict__ xyz, const double *__restrict__ rad, int N,
                                 const double *__restrict__ dirs, const double *__restrict__ w, int nsph,
                                 const int *__restrict__ keep, int M, const double *__restrict__ r_explicit,
                                 double zeta0, double diag_const, double *__restrict__ px, double *__restrict__ py,
                                 double *__restrict__ pz, double *__restrict__ zeta_o, double *__restrict__ S_o,
                                 double *__restrict__ Akk, int Mpad, PtInt<double> *__restrict__ pti64,
                                 PtInt<float> *__restrict__ pti32, double *__restrict__ qpad) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mpad) return;
    if (k >= M) {  // far-away dummy points (zero charge) completing the last batch
        pti64[k] = PtInt<double>{1e6, 1e6, 1e6, 1.0, 1.0, BoysCfg<double>::TMAX};
        pti32[k] = PtInt<float>{1e6, 1e6, 1e6, 1.0f, 1.0f, BoysCfg<float>::TMAX};
        qpad[k] = 0.0;
        return;
    }
    int kr = keep[k];
    int I = kr / nsph, j = kr - I * nsph;
    double zeta = zeta0 / (rad[I] * sqrt(w[j]));
    double x, y, z;
    if (r_explicit) {
        x = r_explicit[3 * k]; y = r_explicit[3 * k + 1]; z = r_explicit[3 * k + 2];
    } else {
        x = xyz[3 * I] + rad[I] * dirs[3 * j];
        y = xyz[3 * I + 1] + rad[I] * dirs[3 * j + 1];
        z = xyz[3 * I + 2] + rad[I] * dirs[3 * j + 2];
    }
    double s = switching_product(xyz, rad, N, I, x, y, z, zeta);
    px[k] = x; py[k] = y; pz[k] = z;
    zeta_o[k] = zeta;
    S_o[k] = s;
    Akk[k] = diag_const * zeta / s;
    double z2 = zeta * zeta;
    pti64[k] = PtInt<double>{x, y, z, z2, zeta, BoysCfg<double>::TMAX / z2};
    pti32[k] = PtInt<float>{x, y, z, (float)z2, (float)zeta, (float)((double)BoysCfg<float>::TMAX / z2)};
}

void surface_build(pcm_ctx *ctx, pcm_mol *mol, bool prune) {
    const int T = 256;
    if (prune) {
        int nraw = mol->N * mol->nsph;
        mol->Mraw = nraw;
        DevBuf<int> flag, pos;
        flag.ensure(nraw);
        pos.ensure(nraw);
        k_surface_flags<<<div_up(nraw, T), T, 0, ctx->stream>>>(mol->xyz.p, mol->rad.p, mol->N, mol->dirs.p, mol->w.p,
                                                                 mol->nsph, ctx->prm.zeta0, ctx->prm.switch_thresh,
                                                                 flag.p);
        HIP_LAUNCH_OK();
        long long M = 0;
        scan_exclusive(ctx, mol, flag.p, pos.p, nraw, &M);
        mol->M = (int)M;
        if (M == 0) {
            flag.release();
            pos.release();
            throw PcmError{PCM_E_ARG, "every surface point is buried (S_k < switch_thresh)"};
        }
        mol->keep.ensure(M);
        k_surface_compact<<<div_up(nraw, T), T, 0, ctx->stream>>>(flag.p, pos.p, nraw, mol->keep.p);
        HIP_LAUNCH_OK();
        mol->h_keep.resize(M);
        HIP_OK(hipMemcpyAsync(mol->h_keep.data(), mol->keep.p, M * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        flag.release();
        pos.release();
        int Mi = mol->M;
        mol->px.ensure(Mi); mol->py.ensure(Mi); mol->pz.ensure(Mi);
        mol->zeta.ensure(Mi); mol->S.ensure(Mi); mol->Akk.ensure(Mi);
        mol->Mpad = (Mi + PT_PAD - 1) / PT_PAD * PT_PAD;
        mol->pti64.ensure(sizeof(PtInt<double>) * (size_t)mol->Mpad);
        mol->pti32.ensure(sizeof(PtInt<float>) * (size_t)mol->Mpad);
        mol->qpad.ensure(mol->Mpad);
    }
}

// Order in which the point-per-lane kernels take the surface points: along a Morton curve of
// their positions (30 bits on a 1024^3 grid over the cavity), so that a wave's points are close
// together and fewer waves take the near-field branch for a pair.  Results do not depend on it.
__global__ void k_point_key(int M, const double *__restrict__ px, const double *__restrict__ py,
                            const double *__restrict__ pz, double lox, double loy, double loz, double inv_cell,
                            unsigned *__restrict__ key, int *__restrict__ val) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const double r[3] = {px[k] - lox, py[k] - loy, pz[k] - loz};
    unsigned m = 0;
    for (int d = 0; d < 3; ++d) {
        const int g = min(1023, max(0, (int)(r[d] * inv_cell)));
        for (int bit = 0; bit < 10; ++bit) m |= (unsigned)((g >> bit) & 1) << (3 * bit + d);
    }
    key[k] = m;
    val[k] = k;
}

static void points_order(pcm_ctx *ctx, pcm_mol *mol) {
    const int M = mol->M;
    mol->pperm.ensure(M + 1);
    if (M <= 0) return;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, rmax = 0.0;
    for (int i = 0; i < mol->N; ++i) {
        rmax = std::max(rmax, mol->h_rad[i]);
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], mol->h_xyz[3 * i + d]);
            hi[d] = std::max(hi[d], mol->h_xyz[3 * i + d]);
        }
    }
    const double pad = 2.0 * rmax + 1.0;  // covers points moved or given explicitly nearby
    for (int d = 0; d < 3; ++d) {
        lo[d] -= pad;
        hi[d] += pad;
    }
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    mol->okey.ensure(2 * (size_t)M);
    mol->oval.ensure(M);
    k_point_key<<<div_up(M, 256), 256, 0, ctx->stream>>>(M, mol->px.p, mol->py.p, mol->pz.p, lo[0], lo[1], lo[2],
                                                         1023.999 / ext, mol->okey.p, mol->oval.p);
    HIP_LAUNCH_OK();
    size_t bytes = 0;
    HIP_OK(rocprim::radix_sort_pairs(nullptr, bytes, mol->okey.p, mol->okey.p + M, mol->oval.p, mol->pperm.p, M, 0,
                                     30, ctx->stream));
    mol->osort.ensure(bytes + 1);
    HIP_OK(rocprim::radix_sort_pairs(mol->osort.p, bytes, mol->okey.p, mol->okey.p + M, mol->oval.p, mol->pperm.p,
                                     M, 0, 30, ctx->stream));
}

void surface_points(pcm_ctx *ctx, pcm_mol *mol, const double *r_explicit_dev) {
    const int T = 256;
    k_surface_points<<<grid_for(mol->Mpad, T), T, 0, ctx->stream>>>(
        mol->xyz.p, mol->rad.p, mol->N, mol->dirs.p, mol->w.p, mol->nsph, mol->keep.p, mol->M, r_explicit_dev,
        ctx->prm.zeta0, ctx->prm.diag_const, mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p, mol->S.p, mol->Akk.p,
        mol->Mpad, reinterpret_cast<PtInt<double> *>(mol->pti64.p), reinterpret_cast<PtInt<float> *>(mol->pti32.p),
        mol->qpad.p);
    HIP_LAUNCH_OK();
    points_order(ctx, mol);
}

// ----------------------------------------------------------------------------------------
// Basis normalisation (Eqs. 11-12): every Cartesian component of a contracted shell gets
// unit self-overlap.  cn[cnoff[s] + c*np + i] = d_i N_i(c) / sqrt(<phi_c|phi_c>).
// ----------------------------------------------------------------------------------------
__device__ double dfact_odd(int n) {
    double r = 1.0;
    for (int k = 2 * n - 1; k > 1; k -= 2) r *= (double)k;
    return r;
}

__global__ void k_normalise(int ns, const int *__restrict__ sl, const int *__restrict__ snp,
                            const int *__restrict__ soff, const int *__restrict__ cnoff,
                            const double *__restrict__ pexp, const double *__restrict__ pcoef,
                            double *__restrict__ cn) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    int l = sl[s], np = snp[s];
    for (int c = 0; c < ncart(l); ++c) {
        int ax, ay, az;
        cart_comp(l, c, ax, ay, az);
        double df = dfact_odd(ax) * dfact_odd(ay) * dfact_odd(az);
        double tmp[8];
        for (int i = 0; i < np; ++i) {
            double a = pexp[soff[s] + i];
            double t = 2.0 * a / M_PI;
            double g = 1.0;
            for (int k = 0; k < l; ++k) g *= 4.0 * a;
            tmp[i] = pcoef[soff[s] + i] * sqrt(t * sqrt(t) * g / df);
        }
        double ov = 0.0;
        for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j) {
                double p = pexp[soff[s] + i] + pexp[soff[s] + j];
                double t = M_PI / p;
                double g = 1.0;
                for (int k = 0; k < l; ++k) g *= 2.0 * p;
                ov += tmp[i] * tmp[j] * (t * sqrt(t)) * df / g;
            }
        double sc = 1.0 / sqrt(ov);
        for (int i = 0; i < np; ++i) cn[cnoff[s] + c * np + i] = tmp[i] * sc;
    }
}

void basis_normalise(pcm_ctx *ctx, pcm_mol *mol) {
    k_normalise<<<div_up(mol->ns, 128), 128, 0, ctx->stream>>>(mol->ns, mol->sl.p, mol->snp.p, mol->soff.p,
                                                                mol->cnoff.p, mol->pexp.p, mol->pcoef.p, mol->cn.p);
    HIP_LAUNCH_OK();
}

// ----------------------------------------------------------------------------------------
// Primitive-pair screening (Sec. 4a, Eq. 15; Eq. 18 with the density).  The bound of a
// primitive pair is the exact [ij|ij]^(1/2) of the s-type product with the same exponents,
// times |c_i c_j| (normalised coefficients of the x^l component):
//   |c_i c_j| sqrt(2 pi^(5/2) / (p^2 sqrt(2p))) exp(-a b / p |A-B|^2);
// with P it is further multiplied by max |P_{mu nu}| over the shell-pair block.
// ----------------------------------------------------------------------------------------
__global__ void k_screen(int nsp, const int *__restrict__ spa, const int *__restrict__ spb,
                         const int *__restrict__ sl, const int *__restrict__ snp, const int *__restrict__ soff,
                         const int *__restrict__ satom, const int *__restrict__ bfo, const int *__restrict__ cnoff,
                         const double *__restrict__ pexp, const double *__restrict__ cn,
                         const double *__restrict__ xyz, const double *__restrict__ P, int nbf, double c2,
                         double thresh, unsigned long long *__restrict__ mask, int *__restrict__ cnt) {
    int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nsp) return;
    int a = spa[sp], b = spb[sp];
    double pm = 1.0;
    if (P) {
        pm = 0.0;
        int na = ncart(sl[a]), nb = ncart(sl[b]);
        for (int mu = 0; mu < na; ++mu)
            for (int nu = 0; nu < nb; ++nu) {
                double v = fabs(P[(long long)(bfo[a] + mu) * nbf + bfo[b] + nu]);
                pm = v > pm ? v : pm;
            }
    }
    const double *A = xyz + 3 * satom[a], *B = xyz + 3 * satom[b];
    double ab2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    unsigned long long m = 0;
    int n = 0;
    for (int i = 0; i < snp[a]; ++i)
        for (int j = 0; j < snp[b]; ++j) {
            double ea = pexp[soff[a] + i], eb = pexp[soff[b] + j], p = ea + eb;
            double ci = fabs(cn[cnoff[a] + i]), cj = fabs(cn[cnoff[b] + j]);
            double bound = ci * cj * sqrt(c2 / (p * p * sqrt(2.0 * p))) * exp(-ea * eb / p * ab2);
            if (pm * bound >= thresh) {
                m |= 1ull << (i * 8 + j);
                ++n;
            }
        }
    mask[sp] = m;
    cnt[sp] = n;
}

__global__ void k_screen_write(int nsp, const unsigned long long *__restrict__ mask, const int *__restrict__ spo,
                               int *__restrict__ ent_sp, int *__restrict__ ent_ij) {
    int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nsp) return;
    unsigned long long m = mask[sp];
    int o = spo[sp];
    for (int bit = 0; bit < 64; ++bit)
        if (m >> bit & 1ull) {
            ent_sp[o] = sp;
            ent_ij[o] = bit;
            ++o;
        }
}

__global__ void k_zero_int(int *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

static void screen_launch(pcm_ctx *ctx, pcm_mol *mol, const double *P, double thresh, unsigned long long *mask,
                          int *cnt) {
    const long long nsp = mol->sp_cls_off[NCLS];
    if (nsp <= 0) return;
    const int T = 256;
    const double c2 = 2.0 * pow(M_PI, 2.5);
    k_screen<<<div_up(nsp, T), T, 0, ctx->stream>>>((int)nsp, mol->spa.p, mol->spb.p, mol->sl.p, mol->snp.p,
                                                     mol->soff.p, mol->satom.p, mol->bfo.p, mol->cnoff.p, mol->pexp.p,
                                                     mol->cn.p, mol->xyz.p, P, mol->nbf, c2, thresh, mask, cnt);
    HIP_LAUNCH_OK();
}

// Order of the records for the pair-per-lane kernels: key = class (3 bits), exponent octave of
// p = a + b (4 bits: p from 1/4 to 2^14), Morton code of the product centre on a 256^3 grid over
// the molecule (24 bits); value = the class-local record index.
struct ClsBounds {
    long long o[NCLS + 1];
};
__global__ void k_pair_key(long long n, ClsBounds cb, const int *__restrict__ ent_sp, const int *__restrict__ ent_ij,
                           const int *__restrict__ spa, const int *__restrict__ spb, const int *__restrict__ soff,
                           const int *__restrict__ satom, const double *__restrict__ pexp,
                           const double *__restrict__ xyz, double lox, double loy, double loz, double inv_cell,
                           unsigned *__restrict__ key, int *__restrict__ val) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int c = 0;
    while (c < NCLS - 1 && q >= cb.o[c + 1]) ++c;
    const int sp = ent_sp[q], ij = ent_ij[q];
    const int a = spa[sp], b = spb[sp];
    const double ea = pexp[soff[a] + (ij >> 3)], eb = pexp[soff[b] + (ij & 7)], p = ea + eb;
    const double *A = xyz + 3 * satom[a], *B = xyz + 3 * satom[b];
    const double P[3] = {(ea * A[0] + eb * B[0]) / p, (ea * A[1] + eb * B[1]) / p, (ea * A[2] + eb * B[2]) / p};
    const double lo[3] = {lox, loy, loz};
    unsigned m = 0;
    for (int d = 0; d < 3; ++d) {
        const int g = min(255, max(0, (int)((P[d] - lo[d]) * inv_cell)));
        for (int bit = 0; bit < 8; ++bit) m |= (unsigned)((g >> bit) & 1) << (3 * bit + d);
    }
    const int oct = min(15, max(0, (int)floor(log2(p)) + 2));
    key[q] = ((unsigned)c << 28) | ((unsigned)oct << 24) | m;
    val[q] = (int)(q - cb.o[c]);
}

static void pairs_order(pcm_ctx *ctx, pcm_mol *mol, PairList &pl) {
    const long long n = pl.n;
    pl.vperm.ensure(n + 1);
    if (n == 0) return;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < mol->N; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], mol->h_xyz[3 * i + d]);
            hi[d] = std::max(hi[d], mol->h_xyz[3 * i + d]);
        }
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1.0});
    ClsBounds cb;
    for (int c = 0; c <= NCLS; ++c) cb.o[c] = pl.cls_off[c];
    mol->okey.ensure(2 * (size_t)n);
    mol->oval.ensure(n);
    k_pair_key<<<div_up(n, 256), 256, 0, ctx->stream>>>(n, cb, pl.ent_sp.p, pl.ent_ij.p, mol->spa.p, mol->spb.p,
                                                       mol->soff.p, mol->satom.p, mol->pexp.p, mol->xyz.p, lo[0],
                                                       lo[1], lo[2], 255.999 / ext, mol->okey.p, mol->oval.p);
    HIP_LAUNCH_OK();
    size_t bytes = 0;
    HIP_OK(rocprim::radix_sort_pairs(nullptr, bytes, mol->okey.p, mol->okey.p + n, mol->oval.p, pl.vperm.p, n, 0,
                                     31, ctx->stream));
    mol->osort.ensure(bytes + 1);
    HIP_OK(rocprim::radix_sort_pairs(mol->osort.p, bytes, mol->okey.p, mol->okey.p + n, mol->oval.p, pl.vperm.p, n,
                                     0, 31, ctx->stream));
}

// Per-class metadata of a compacted list in one launch (grid (64, NCLS)): the shell pairs with
// survivors per class (blockIdx.y = class, integer atomics into out[0 .. NCLS), zeroed before, so the
// sums do not depend on their order) and, from block (0, 0), the entry offset of every class boundary
// (out[NCLS .. 2 NCLS]) and the terminating offset spo[nsp] = total.
__global__ void k_list_meta(int nsp, const int *__restrict__ cnt, int *__restrict__ spo, ClsBounds cb,
                            const int *__restrict__ total, int *__restrict__ out) {
    __shared__ int s[256];
    const int c = blockIdx.y;
    const long long b0 = cb.o[c], b1 = cb.o[c + 1];
    int acc = 0;
    for (long long sp = b0 + (long long)blockIdx.x * blockDim.x + threadIdx.x; sp < b1;
         sp += (long long)gridDim.x * blockDim.x)
        acc += cnt[sp] > 0;
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && s[0]) atomicAdd(out + c, s[0]);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x <= NCLS) {
        const long long sb = cb.o[threadIdx.x];
        out[NCLS + threadIdx.x] = sb >= nsp ? *total : spo[sb];
        if (threadIdx.x == 0) spo[nsp] = *total;
    }
}

// entries, per-shell-pair offsets and class offsets of a list from its survivor masks and counts
// (one readback of the class metadata per list)
static void pairs_compact(pcm_ctx *ctx, pcm_mol *mol, PairList &pl) {
    const long long nsp = mol->sp_cls_off[NCLS];
    const int T = 256;
    int meta[2 * NCLS + 1] = {0};
    if (nsp > 0) {
        const int *tot = scan_exclusive_dev(ctx, mol, pl.cnt.p, pl.spo.p, nsp);
        ClsBounds cb;
        for (int c = 0; c <= NCLS; ++c) cb.o[c] = mol->sp_cls_off[c];
        k_zero_int<<<1, 64, 0, ctx->stream>>>(ctx->iscal.p, 2 * NCLS + 1);
        HIP_LAUNCH_OK();
        k_list_meta<<<dim3(64, NCLS), 256, 0, ctx->stream>>>((int)nsp, pl.cnt.p, pl.spo.p, cb, tot, ctx->iscal.p);
        HIP_LAUNCH_OK();
        HIP_OK(hipMemcpyAsync(meta, ctx->iscal.p, sizeof(meta), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    const long long total = meta[2 * NCLS];
    if (total < 0 || total > 2000000000LL) throw PcmError{PCM_E_ALLOC, "screened pair list exceeds 2^31 entries"};
    pl.n = total;
    for (int c = 0; c <= NCLS; ++c) pl.cls_off[c] = meta[NCLS + c];
    for (int c = 0; c < NCLS; ++c) pl.sp_count[c] = meta[c];
    pl.ent_sp.ensure(total + 1);
    pl.ent_ij.ensure(total + 1);
    if (nsp > 0) {
        k_screen_write<<<div_up(nsp, T), T, 0, ctx->stream>>>((int)nsp, pl.mask.p, pl.spo.p, pl.ent_sp.p, pl.ent_ij.p);
        HIP_LAUNCH_OK();
    }
    pairs_order(ctx, mol, pl);
}

void pairs_build(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P, int kind) {
    (void)kind;
    const long long nsp = mol->sp_cls_off[NCLS];
    pl.mask.ensure(nsp + 1);
    pl.cnt.ensure(nsp + 1);
    pl.spo.ensure(nsp + 1);
    screen_launch(ctx, mol, P, ctx->prm.schwarz_thresh, pl.mask.p, pl.cnt.p);
    pairs_compact(ctx, mol, pl);
    for (int c = 0; c < NCLS; ++c) pl.sp_union[c] = pl.sp_count[c];
}

// strong = survivors whose bound also reaches the split threshold; weak = the other survivors
__global__ void k_mask_split(int nsp, const unsigned long long *__restrict__ strong_bits,
                             unsigned long long *__restrict__ mask, int *__restrict__ cnt,
                             unsigned long long *__restrict__ wmask, int *__restrict__ wcnt) {
    int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nsp) return;
    const unsigned long long all = mask[sp], s = all & strong_bits[sp], w = all & ~s;
    mask[sp] = s;
    cnt[sp] = __popcll(s);
    wmask[sp] = w;
    wcnt[sp] = __popcll(w);
}

void pairs_split(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, PairList &weak, const double *P, double thresh) {
    const long long nsp = mol->sp_cls_off[NCLS];
    weak.mask.ensure(nsp + 1);
    weak.cnt.ensure(nsp + 1);
    weak.spo.ensure(nsp + 1);
    if (nsp > 0) {
        mol->mtmp.ensure(3 * (size_t)nsp);
        mol->ctmp.ensure(nsp);
        screen_launch(ctx, mol, P, std::max(thresh, ctx->prm.schwarz_thresh), mol->mtmp.p, mol->ctmp.p);
        k_mask_split<<<div_up(nsp, 256), 256, 0, ctx->stream>>>((int)nsp, mol->mtmp.p, pl.mask.p, pl.cnt.p,
                                                                weak.mask.p, weak.cnt.p);
        HIP_LAUNCH_OK();
    }
    pairs_compact(ctx, mol, pl);
    pairs_compact(ctx, mol, weak);
}

// ----------------------------------------------------------------------------------------
// Pair records.  Header: P, p, TMAX/p, (pi/p)^{3/2} K, (2 pi/p) K with K = exp(-ab/p |A-B|^2).
// For density lists the header is followed by D_tuv = -w sum_{mu in a, nu in b} P_{mu nu}
// c_{mu i} c_{nu j} E^{mu nu}_tuv (w = 2 for a != b, Eqs. 5-6 with P symmetric).
// ----------------------------------------------------------------------------------------
template <typename T>
__device__ void pair_header(int sp, int ij, const int *__restrict__ spa, const int *__restrict__ spb,
                            const int *__restrict__ soff, const int *__restrict__ satom,
                            const double *__restrict__ pexp, const double *__restrict__ xyz, PairHdr<T> &h,
                            double &PAx, double &PAy, double &PAz, double &PBx, double &PBy, double &PBz,
                            double &p_out) {
    int a = spa[sp], b = spb[sp];
    int i = ij >> 3, j = ij & 7;
    double ea = pexp[soff[a] + i], eb = pexp[soff[b] + j];
    const double *A = xyz + 3 * satom[a], *B = xyz + 3 * satom[b];
    double p = ea + eb;
    double Px = (ea * A[0] + eb * B[0]) / p, Py = (ea * A[1] + eb * B[1]) / p, Pz = (ea * A[2] + eb * B[2]) / p;
    double ab2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    double K = exp(-ea * eb / p * ab2);
    double t = M_PI / p;
    h.Px = Px; h.Py = Py; h.Pz = Pz;
    h.p = (T)p;
    h.limp = (T)((double)BoysCfg<T>::TMAX / p);
    h.pf = (T)(t * sqrt(t) * K);
    h.pref = (T)(2.0 * M_PI / p * K);
    PAx = Px - A[0]; PAy = Py - A[1]; PAz = Pz - A[2];
    PBx = Px - B[0]; PBy = Py - B[1]; PBz = Pz - B[2];
    p_out = p;
}

template <int LA, int LB, typename T>
__global__ void k_prep_geom(long long n, const int *__restrict__ ent_sp, const int *__restrict__ ent_ij,
                            const int *__restrict__ spa, const int *__restrict__ spb, const int *__restrict__ soff,
                            const int *__restrict__ satom, const double *__restrict__ pexp,
                            const double *__restrict__ xyz, unsigned char *__restrict__ rec, size_t stride) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    PairHdr<T> h;
    double a0, a1, a2, b0, b1, b2, p;
    pair_header<T>(ent_sp[q], ent_ij[q], spa, spb, soff, satom, pexp, xyz, h, a0, a1, a2, b0, b1, b2, p);
    *reinterpret_cast<PairHdr<T> *>(rec + q * stride) = h;
}

template <int LA, int LB, typename T>
__global__ void k_prep_density(long long n, const int *__restrict__ ent_sp, const int *__restrict__ ent_ij,
                               const int *__restrict__ spa, const int *__restrict__ spb, const int *__restrict__ snp,
                               const int *__restrict__ soff, const int *__restrict__ satom,
                               const int *__restrict__ bfo, const int *__restrict__ cnoff,
                               const double *__restrict__ pexp, const double *__restrict__ cn,
                               const double *__restrict__ xyz, const double *__restrict__ P, int nbf,
                               unsigned char *__restrict__ rec, size_t stride) {
    constexpr int L = LA + LB;
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int sp = ent_sp[q], ij = ent_ij[q];
    PairHdr<T> h;
    double PA[3], PB[3], p;
    pair_header<T>(sp, ij, spa, spb, soff, satom, pexp, xyz, h, PA[0], PA[1], PA[2], PB[0], PB[1], PB[2], p);
    int a = spa[sp], b = spb[sp];
    int i = ij >> 3, j = ij & 7;
    double inv2p = 0.5 / p;
    Herm1D<LA, LB> ex, ey, ez;
    ex.build(PA[0], PB[0], inv2p);
    ey.build(PA[1], PB[1], inv2p);
    ez.build(PA[2], PB[2], inv2p);
    double w = (a == b) ? -1.0 : -2.0;
    double D[ntuv(L)];
    for (int t = 0; t < ntuv(L); ++t) D[t] = 0.0;
    for (int mu = 0; mu < ncart(LA); ++mu) {
        int ax, ay, az;
        cart_comp(LA, mu, ax, ay, az);
        double cmu = cn[cnoff[a] + mu * snp[a] + i];
        for (int nu = 0; nu < ncart(LB); ++nu) {
            int bx, by, bz;
            cart_comp(LB, nu, bx, by, bz);
            double cf = w * P[(long long)(bfo[a] + mu) * nbf + bfo[b] + nu] * cmu * cn[cnoff[b] + nu * snp[b] + j];
            for (int t = 0; t <= ax + bx; ++t)
                for (int u = 0; u <= ay + by; ++u) {
                    double ctu = cf * ex.e[ax][bx][t] * ey.e[ay][by][u];
                    for (int v = 0; v <= az + bz; ++v) D[tuv_idx(t, u, v)] += ctu * ez.e[az][bz][v];
                }
        }
    }
    unsigned char *r = rec + q * stride;
    *reinterpret_cast<PairHdr<T> *>(r) = h;
    T *Dd = reinterpret_cast<T *>(r + sizeof(PairHdr<T>));
    for (int t = 0; t < ntuv(L); ++t) Dd[t] = (T)D[t];
}

// zero-contribution records completing the last batch of a class: far away, D = 0
template <typename T>
__global__ void k_zero_records(unsigned char *__restrict__ rec, int n, size_t stride, int nt) {
    int q = threadIdx.x;
    if (q >= n) return;
    unsigned char *r = rec + q * stride;
    PairHdr<T> h;
    h.Px = 1e6; h.Py = 1e6; h.Pz = 1e6;
    h.p = T(1); h.limp = BoysCfg<T>::TMAX; h.pf = T(0); h.pref = T(0);
    *reinterpret_cast<PairHdr<T> *>(r) = h;
    T *D = reinterpret_cast<T *>(r + sizeof(PairHdr<T>));
    for (int t = 0; t < nt; ++t) D[t] = T(0);
}

template <typename T>
static void prep_lists_plan(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P, Launches &out) {
    // byte layout: classes back to back, each with its own stride
    size_t off = 0;
    for (int c = 0; c < NCLS; ++c) {
        pl.rec_off[c] = off;
        long long n = pl.cls_off[c + 1] - pl.cls_off[c];
        long long npad = (n + REC_PAD - 1) / REC_PAD * REC_PAD;
        size_t stride = P ? rec_stride<T>(CLS_LA[c] + CLS_LB[c]) : align16(sizeof(PairHdr<T>));
        off += align16(npad * stride) + 256;
    }
    pl.rec_off[NCLS] = off;
    pl.rec.ensure(off);
    const int TB = 128;
    for (int c = 0; c < NCLS; ++c) {
        long long n = pl.cls_off[c + 1] - pl.cls_off[c];
        if (n == 0) continue;
        const int *es = pl.ent_sp.p + pl.cls_off[c], *ei = pl.ent_ij.p + pl.cls_off[c];
        unsigned char *rec = pl.rec.p + pl.rec_off[c];
        int g = div_up(n, TB);
        const int *spa = mol->spa.p, *spb = mol->spb.p, *snp = mol->snp.p, *soff = mol->soff.p,
                  *satom = mol->satom.p, *bfo = mol->bfo.p, *cnoff = mol->cnoff.p;
        const double *pexp = mol->pexp.p, *cn = mol->cn.p, *xyz = mol->xyz.p;
        const int nbf = mol->nbf;
        out.add("", 0.0, [=](hipStream_t st) {
#define PREP_CASE(CI, LA_, LB_)                                                                                     \
    case CI:                                                                                                        \
        if (P)                                                                                                      \
            k_prep_density<LA_, LB_, T><<<g, TB, 0, st>>>(n, es, ei, spa, spb, snp, soff, satom, bfo, cnoff, pexp,  \
                                                          cn, xyz, P, nbf, rec, rec_stride<T>(LA_ + LB_));          \
        else                                                                                                        \
            k_prep_geom<LA_, LB_, T><<<g, TB, 0, st>>>(n, es, ei, spa, spb, soff, satom, pexp, xyz, rec,            \
                                                       align16(sizeof(PairHdr<T>)));                                \
        break;
            switch (c) {
                PREP_CASE(0, 0, 0)
                PREP_CASE(1, 0, 1)
                PREP_CASE(2, 0, 2)
                PREP_CASE(3, 1, 1)
                PREP_CASE(4, 1, 2)
                PREP_CASE(5, 2, 2)
            }
#undef PREP_CASE
            HIP_LAUNCH_OK();
            if (P && n % REC_PAD) {
                size_t stride = rec_stride<T>(CLS_LA[c] + CLS_LB[c]);
                int npad = (int)(REC_PAD - n % REC_PAD);
                k_zero_records<T><<<1, 64, 0, st>>>(rec + n * stride, npad, stride, ntuv(CLS_LA[c] + CLS_LB[c]));
                HIP_LAUNCH_OK();
            }
        });
    }
}

template <typename T>
static void prep_lists(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P) {
    Launches run;
    prep_lists_plan<T>(ctx, mol, pl, P, run);
    run.run(ctx, ctx->stream, false);
}

// the kernels that rebuild a density list's records (header + D_tuv) from the current P; the
// record buffer is laid out now, so the launches themselves allocate nothing
void density_record_launches(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P, int prec, Launches &out) {
    if (prec == PCM_MIXED)
        prep_lists_plan<float>(ctx, mol, pl, P, out);
    else
        prep_lists_plan<double>(ctx, mol, pl, P, out);
}

void pairs_prepare_geometry(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, int prec) {
    if (prec == PCM_MIXED)
        prep_lists<float>(ctx, mol, pl, nullptr);
    else
        prep_lists<double>(ctx, mol, pl, nullptr);
}

void pairs_prepare_density(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P, int prec) {
    if (prec == PCM_MIXED)
        prep_lists<float>(ctx, mol, pl, P);
    else
        prep_lists<double>(ctx, mol, pl, P);
}

// ----------------------------------------------------------------------------------------
// Lists of the one-pass Fock + gradient pair side: the Eq. 18 survivors for P (bits kept in m18),
// whose V' up to L + 1 serves the gradient and the Fock matrix, and the Eq. 15 survivors (bits in
// m15, from fock.mask) outside them, which need V up to L for the Fock matrix only; header-only
// records in the precision of the pass.  Entries keep the list order (class, shell pair, i, j).
// ----------------------------------------------------------------------------------------
__global__ void k_mask_or(int nsp, const unsigned long long *__restrict__ a, const unsigned long long *__restrict__ b,
                          unsigned long long *__restrict__ mask, int *__restrict__ cnt) {
    int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nsp) return;
    const unsigned long long m = a[sp] | b[sp];
    mask[sp] = m;
    cnt[sp] = __popcll(m);
}

// bits of a that are not in b
__global__ void k_mask_andnot(int nsp, const unsigned long long *__restrict__ a, const unsigned long long *__restrict__ b,
                              unsigned long long *__restrict__ mask, int *__restrict__ cnt) {
    int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nsp) return;
    const unsigned long long m = a[sp] & ~b[sp];
    mask[sp] = m;
    cnt[sp] = __popcll(m);
}

void pairs_merged_build(pcm_ctx *ctx, pcm_mol *mol, const double *P, bool dynamic) {
    const long long nsp = mol->sp_cls_off[NCLS];
    PairList &fg = mol->fg, &fgw = mol->fg_w, &fo = mol->fo, &fow = mol->fo_w;
    mol->m18.ensure(nsp + 1);
    mol->c18.ensure(nsp + 1);
    mol->m15.ensure(nsp + 1);
    for (PairList *l : {&fg, &fgw, &fo, &fow}) {
        l->mask.ensure(nsp + 1);
        l->cnt.ensure(nsp + 1);
        l->spo.ensure(nsp + 1);
    }
    if (nsp > 0) {
        const int g = div_up(nsp, 256);
        screen_launch(ctx, mol, P, ctx->prm.schwarz_thresh, mol->m18.p, mol->c18.p);
        // the Eq. 15 bits: the Fock list, or both of its parts when the precision is split
        k_mask_or<<<g, 256, 0, ctx->stream>>>((int)nsp, mol->fock.mask.p, dynamic ? mol->fock_w.mask.p : mol->fock.mask.p,
                                              mol->m15.p, fgw.cnt.p);
        HIP_LAUNCH_OK();
        // fg: the Eq. 18 survivors; fo: the Eq. 15 survivors outside them
        k_mask_or<<<g, 256, 0, ctx->stream>>>((int)nsp, mol->m18.p, mol->m18.p, fg.mask.p, fg.cnt.p);
        HIP_LAUNCH_OK();
        k_mask_andnot<<<g, 256, 0, ctx->stream>>>((int)nsp, mol->m15.p, mol->m18.p, fo.mask.p, fo.cnt.p);
        HIP_LAUNCH_OK();
        if (dynamic) {
            // FP64 parts: entries whose Eq. 15 bound or Eq. 18 weight reaches dp_thresh
            const double th = std::max(ctx->prm.dp_thresh, ctx->prm.schwarz_thresh);
            mol->mtmp.ensure(3 * (size_t)nsp);
            mol->ctmp.ensure(nsp);
            unsigned long long *s1 = mol->mtmp.p, *s2 = s1 + nsp, *s3 = s2 + nsp;
            screen_launch(ctx, mol, nullptr, th, s1, mol->ctmp.p);
            screen_launch(ctx, mol, P, th, s2, mol->ctmp.p);
            k_mask_or<<<g, 256, 0, ctx->stream>>>((int)nsp, s1, s2, s3, mol->ctmp.p);
            HIP_LAUNCH_OK();
            k_mask_split<<<g, 256, 0, ctx->stream>>>((int)nsp, s3, fg.mask.p, fg.cnt.p, fgw.mask.p, fgw.cnt.p);
            HIP_LAUNCH_OK();
            k_mask_split<<<g, 256, 0, ctx->stream>>>((int)nsp, s3, fo.mask.p, fo.cnt.p, fow.mask.p, fow.cnt.p);
            HIP_LAUNCH_OK();
        }
    }
    for (PairList *l : {&fg, &fo}) {
        pairs_compact(ctx, mol, *l);
        for (int c = 0; c < NCLS; ++c) l->sp_union[c] = l->sp_count[c];
        pairs_prepare_geometry(ctx, mol, *l, PCM_FP64);
    }
    for (PairList *l : {&fgw, &fow}) {
        if (dynamic) {
            pairs_compact(ctx, mol, *l);
            pairs_prepare_geometry(ctx, mol, *l, PCM_MIXED);  // FP32 records
        } else {
            l->n = 0;
            for (int c = 0; c <= NCLS; ++c) l->cls_off[c] = 0;
        }
    }
}
