// Linear solve of Sec. 2, Eq. 1 (A q = -f (Bz + c)) on gfx950.
//
//  * A x is applied matrix-free (A is never stored): A_kl = erf(zeta'_kl r)/r (Eqs. 2, 8) for
//    k != l, A_kk from Eq. 3.  One lane per row k; the wave walks a chunk of columns l whose
//    data are wave-uniform.  erf(zeta' r) rounds to 1 once zeta' r >= 6 (FP64) / 4 (FP32):
//    those pairs take the plain 1/r branch, tested with zeta'^2 >= min(zeta_k^2, zeta_l^2)/2.
//  * Preconditioned CG (Sec. 4b) with the residual test ||A q - b||_2 < delta (Eq. 20);
//    Jacobi or randomized block-Jacobi (Sec. 4b-ii) preconditioners; the block inverses are
//    built on the device and applied as a batched GEMV (HBM-bound).
//  * Mixed precision: FP32 matvec inside FP64 iterative refinement; FP64 vectors, dots and
//    the outer residual.
//  * Every reduction is a fixed-order tree: results are bitwise reproducible.
#include "pcm_internal.h"

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>

constexpr int MV_T = 256;
constexpr int MV_B = 8;  // columns per batch of wave-uniform loads

// ----------------------------------------------------------------------------------------
// matrix-free off-diagonal product, partial over a chunk of columns.  Point arrays are
// padded to a multiple of 64 with far-away dummy points whose x entries are zero, so the
// column loop runs over whole batches of 8.
// ----------------------------------------------------------------------------------------
template <typename T> struct Pt {
    T x, y, z, zeta;
};

inline int mv_pad(int M) { return (M + 63) & ~63; }

__global__ void k_pack_pts(const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ pz,
                           const double *__restrict__ zeta, int M, int Mp, Pt<double> *__restrict__ p64,
                           Pt<float> *__restrict__ p32, double *__restrict__ x64, float *__restrict__ x32) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mp) return;
    if (k < M) {
        p64[k] = Pt<double>{px[k], py[k], pz[k], zeta[k]};
        p32[k] = Pt<float>{(float)px[k], (float)py[k], (float)pz[k], (float)zeta[k]};
    } else {
        p64[k] = Pt<double>{1e6, 1e6, 1e6, 1.0};
        p32[k] = Pt<float>{1e6f, 1e6f, 1e6f, 1.0f};
        x64[k] = 0.0;
        x32[k] = 0.0f;
    }
}

template <typename T>
__global__ void k_pad_x(const double *__restrict__ x, T *__restrict__ y, int M) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) y[k] = (T)x[k];
}

__device__ __forceinline__ double erf_t(double x) { return erf(x); }
__device__ __forceinline__ float erf_t(float x) { return erff(x); }

// A_kl inside the cutoff radius (erf not yet 1): coincident points take 2 z'/sqrt(pi)
template <typename T>
__device__ __attribute__((noinline)) T mv_near(T zk, T zl, T r2, bool self) {
    if (self) return T(0);
    T zp = zk * zl * rsqrt_t(zk * zk + zl * zl);
    if (r2 == T(0)) return T(1.1283791670955125739) * zp;
    T r = sqrt_t(r2);
    return erf_t(zp * r) / r;
}

template <typename T>
__global__ __launch_bounds__(MV_T) void k_matvec(const Pt<T> *__restrict__ pts, const T *__restrict__ xv, int M,
                                                 int ncol, int chunk_len, T rc2, double *__restrict__ part) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = k < M ? k : M - 1;
    const Pt<T> me = pts[kk];
    const int l0 = blockIdx.y * chunk_len;
    const int l1 = min(ncol, l0 + chunk_len);
    T acc = T(0);
    for (int l = l0; l < l1; l += MV_B) {
        Pt<T> o[MV_B];
        T xl[MV_B], a[MV_B], r2[MV_B];
#pragma unroll
        for (int u = 0; u < MV_B; ++u) {
            o[u] = pts[l + u];
            xl[u] = xv[l + u];
        }
        bool near = false;
#pragma unroll
        for (int u = 0; u < MV_B; ++u) {
            T dx = me.x - o[u].x, dy = me.y - o[u].y, dz = me.z - o[u].z;
            r2[u] = fma(dx, dx, fma(dy, dy, dz * dz));
            near |= r2[u] < rc2;
            a[u] = rsq_fast(r2[u]);
        }
        if (near) {
#pragma unroll
            for (int u = 0; u < MV_B; ++u)
                if (r2[u] < rc2) a[u] = mv_near<T>(me.zeta, o[u].zeta, r2[u], l + u == kk);
        }
#pragma unroll
        for (int u = 0; u < MV_B; ++u) acc = fma(a[u], xl[u], acc);
    }
    if (k < M) part[(size_t)blockIdx.y * M + k] = (double)acc;
}

// y = Akk x + sum of partial rows; optionally the per-block partial of sum_k x_k y_k
__global__ __launch_bounds__(256) void k_mv_finish(const double *__restrict__ part, int rows, int M,
                                                   const double *__restrict__ Akk, const double *__restrict__ x,
                                                   double *__restrict__ y, double *__restrict__ dotpart) {
    __shared__ double s[256];
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0;
    if (k < M) {
        double acc = Akk[k] * x[k];
        double off = 0.0;
        for (int r = 0; r < rows; ++r) off += part[(size_t)r * M + k];
        acc += off;
        y[k] = acc;
        d = x[k] * acc;
    }
    if (dotpart) {
        s[threadIdx.x] = d;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) dotpart[blockIdx.x] = s[0];
    }
}

static int mv_chunk_len(int Mp) {
    int tiles = div_up(Mp, MV_T);
    int want = div_up(2048, tiles);
    int len = div_up(Mp, want);
    len = (len + MV_B - 1) / MV_B * MV_B;
    return len < 64 ? 64 : len;
}

// solver workspace layout inside mol->sv (offsets in doubles, each slot 32-aligned)
struct SolverLayout {
    size_t r, z, p, Ap, y, dp1, dp2, dp3, b, d, res, dot, p64, p32, x64, x32, total;
};

static SolverLayout solver_layout(size_t M) {
    SolverLayout L{};
    size_t o = 0, Mp = mv_pad((int)M);
    auto take = [&](size_t n) {
        size_t s0 = o;
        o += (n + 31) & ~size_t(31);
        return s0;
    };
    L.r = take(M); L.z = take(M); L.p = take(M); L.Ap = take(M); L.y = take(M);
    L.dp1 = take(2 * M + 4096); L.dp2 = take(2 * M + 4096); L.dp3 = take(2 * M + 4096);
    L.b = take(M); L.d = take(M); L.res = take(M); L.dot = take(M / 256 + 64);
    L.p64 = take(4 * Mp); L.p32 = take(2 * Mp); L.x64 = take(Mp); L.x32 = take(Mp / 2 + 2);
    L.total = o;
    return L;
}

struct MatvecWS {
    Pt<double> *p64;
    Pt<float> *p32;
    double *x64;
    float *x32;
};

static MatvecWS mv_ws(pcm_mol *mol) {
    SolverLayout L = solver_layout(mol->M);
    MatvecWS w;
    w.p64 = reinterpret_cast<Pt<double> *>(mol->sv.p + L.p64);
    w.p32 = reinterpret_cast<Pt<float> *>(mol->sv.p + L.p32);
    w.x64 = mol->sv.p + L.x64;
    w.x32 = reinterpret_cast<float *>(mol->sv.p + L.x32);
    return w;
}

// cutoff radius^2 beyond which erf(z' r) rounds to 1 for every pair: z'^2 >= zeta_min^2 / 2
static void mv_cutoffs(pcm_mol *mol, double &rc2_64, double &rc2_32) {
    double zmin = 1e300;
    for (int kr : mol->h_keep) {
        int I = kr / mol->nsph, j = kr - I * mol->nsph;
        zmin = std::min(zmin, mol->zeta0 / (mol->h_rad[I] * std::sqrt(mol->h_w[j])));
    }
    zmin *= 1.0 - 1e-9;
    rc2_64 = 2.0 * 36.0 / (zmin * zmin);
    rc2_32 = 2.0 * 16.0 / (zmin * zmin);
}

static void ensure_solver_ws(pcm_ctx *ctx, pcm_mol *mol) {
    size_t M = mol->M;
    int Mp = mv_pad((int)M);
    mol->sv.ensure(solver_layout(M).total);
    MatvecWS w = mv_ws(mol);
    k_pack_pts<<<div_up(Mp, 256), 256, 0, ctx->stream>>>(mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p, (int)M, Mp,
                                                         w.p64, w.p32, w.x64, w.x32);
    HIP_LAUNCH_OK();
}

// y = A x (FP64 or FP32 off-diagonal); dotpart (may be null) receives per-block x.y partials
static void matvec(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int prec, double *dotpart) {
    const int M = mol->M, Mp = mv_pad(M);
    MatvecWS w = mv_ws(mol);
    int len = mv_chunk_len(Mp);
    int rows = div_up(Mp, len);
    mol->part2.ensure((size_t)rows * M);
    dim3 grid(div_up(M, MV_T), rows);
    double rc64, rc32;
    mv_cutoffs(mol, rc64, rc32);
    if (prec == PCM_MIXED) {
        k_pad_x<float><<<div_up(M, 256), 256, 0, ctx->stream>>>(x, w.x32, M);
        HIP_LAUNCH_OK();
        ProfScope ps(ctx, "matvec_f32", (double)M * M);
        k_matvec<float><<<grid, MV_T, 0, ctx->stream>>>(w.p32, w.x32, M, Mp, len, (float)rc32, mol->part2.p);
        HIP_LAUNCH_OK();
    } else {
        k_pad_x<double><<<div_up(M, 256), 256, 0, ctx->stream>>>(x, w.x64, M);
        HIP_LAUNCH_OK();
        ProfScope ps(ctx, "matvec_f64", (double)M * M);
        k_matvec<double><<<grid, MV_T, 0, ctx->stream>>>(w.p64, w.x64, M, Mp, len, rc64, mol->part2.p);
        HIP_LAUNCH_OK();
    }
    k_mv_finish<<<div_up(M, 256), 256, 0, ctx->stream>>>(mol->part2.p, rows, M, mol->Akk.p, x, y, dotpart);
    HIP_LAUNCH_OK();
}

void run_matvec(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int prec) {
    ensure_solver_ws(ctx, mol);
    matvec(ctx, mol, x, y, prec, nullptr);
}

// ----------------------------------------------------------------------------------------
// deterministic dot products
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dot_part(const double *__restrict__ a, const double *__restrict__ b,
                                                  long long n, double *__restrict__ part) {
    __shared__ double s[256];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    s[threadIdx.x] = i < n ? a[i] * b[i] : 0.0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// sum of nparts partials by one block (fixed order), written to out[0]
__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int nparts,
                                                   double *__restrict__ out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

__device__ __forceinline__ double block_sum_parts(const double *__restrict__ part, int nparts, double *s) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    double r = s[0];
    __syncthreads();
    return r;
}

double dev_dot(pcm_ctx *ctx, pcm_mol *mol, const double *a, const double *b, long long n) {
    int nb = div_up(n, 256);
    double *part = mol->sv.p + solver_layout(mol->M).dot;
    k_dot_part<<<nb, 256, 0, ctx->stream>>>(a, b, n, part);
    HIP_LAUNCH_OK();
    k_sum_parts<<<1, 256, 0, ctx->stream>>>(part, nb, ctx->scal.p);
    HIP_LAUNCH_OK();
    double r = 0.0;
    HIP_OK(hipMemcpyAsync(&r, ctx->scal.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return r;
}

// ----------------------------------------------------------------------------------------
// PCG building blocks.  Scalars live on the device in hist[it][*]:
//   0: p.Ap   1: alpha   2: r.r (after the update)   3: r.z   4: beta
// ----------------------------------------------------------------------------------------
constexpr int HS = 8;

// x += alpha p, r -= alpha Ap, z = r / Akk (jacobi) or z = r (none); partials of r.r and r.z
__global__ __launch_bounds__(256) void k_cg_update(int M, const double *__restrict__ dp_pAp, int n_dp,
                                                   double *__restrict__ hist, int it, double *__restrict__ x,
                                                   double *__restrict__ r, const double *__restrict__ p,
                                                   const double *__restrict__ Ap, double *__restrict__ z,
                                                   const double *__restrict__ Akk, int precond,
                                                   double *__restrict__ dp_rr, double *__restrict__ dp_rz) {
    __shared__ double s[256];
    double pAp = block_sum_parts(dp_pAp, n_dp, s);
    double rz_old = hist[(it - 1) * HS + 3];
    double alpha = rz_old / pAp;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hist[it * HS + 0] = pAp;
        hist[it * HS + 1] = alpha;
    }
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, rz = 0.0;
    if (k < M) {
        x[k] += alpha * p[k];
        double rk = r[k] - alpha * Ap[k];
        r[k] = rk;
        rr = rk * rk;
        if (precond != PCM_PRECOND_RBJ) {
            double zk = precond == PCM_PRECOND_JACOBI ? rk / Akk[k] : rk;
            z[k] = zk;
            rz = rk * zk;
        }
    }
    s[threadIdx.x] = rr;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) dp_rr[blockIdx.x] = s[0];
    __syncthreads();
    s[threadIdx.x] = rz;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && precond != PCM_PRECOND_RBJ) dp_rz[blockIdx.x] = s[0];
}

// reduce r.r (n_rr partials) and r.z (n_rz partials); beta = rz_new / rz_old; p = z + beta p
__global__ __launch_bounds__(256) void k_cg_direction(int M, const double *__restrict__ dp_rr, int n_rr,
                                                      const double *__restrict__ dp_rz, int n_rz,
                                                      double *__restrict__ hist, int it, double *__restrict__ p,
                                                      const double *__restrict__ z) {
    __shared__ double s[256];
    double rr = block_sum_parts(dp_rr, n_rr, s);
    double rz = block_sum_parts(dp_rz, n_rz, s);
    double beta = rz / hist[(it - 1) * HS + 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hist[it * HS + 2] = rr;
        hist[it * HS + 3] = rz;
        hist[it * HS + 4] = beta;
    }
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) p[k] = z[k] + beta * p[k];
}

// initial: r = b - y (y = A x0 or 0), z = C r (jacobi/none), p = z; partials of r.r, r.z
__global__ __launch_bounds__(256) void k_cg_init(int M, const double *__restrict__ b, const double *__restrict__ y,
                                                 double *__restrict__ r, double *__restrict__ z,
                                                 const double *__restrict__ Akk, int precond,
                                                 double *__restrict__ dp_rr, double *__restrict__ dp_rz) {
    __shared__ double s[256];
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, rz = 0.0;
    if (k < M) {
        double rk = b[k] - (y ? y[k] : 0.0);
        r[k] = rk;
        rr = rk * rk;
        if (precond != PCM_PRECOND_RBJ) {
            double zk = precond == PCM_PRECOND_JACOBI ? rk / Akk[k] : rk;
            z[k] = zk;
            rz = rk * zk;
        }
    }
    s[threadIdx.x] = rr;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) dp_rr[blockIdx.x] = s[0];
    __syncthreads();
    s[threadIdx.x] = rz;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && precond != PCM_PRECOND_RBJ) dp_rz[blockIdx.x] = s[0];
}

__global__ void k_axpy(int M, double a, const double *__restrict__ x, double *__restrict__ y) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) y[k] += a * x[k];
}

__global__ void k_scale_copy(int M, double a, const double *__restrict__ x, double *__restrict__ y) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) y[k] = a * x[k];
}

// ----------------------------------------------------------------------------------------
// randomized block-Jacobi: block matrices, in-place SPD inversion, application
// ----------------------------------------------------------------------------------------
__global__ void k_rbj_fill(const Pt<double> *__restrict__ pts, const double *__restrict__ Akk,
                           const int *__restrict__ perm, const int *__restrict__ off, const long long *__restrict__ ioff,
                           double *__restrict__ blk) {
    int b = blockIdx.x;
    int o = off[b], l = off[b + 1] - o;
    long long e = (long long)blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= (long long)l * l) return;
    int i = (int)(e / l), j = (int)(e % l);
    int ki = perm[o + i], kj = perm[o + j];
    double v;
    if (ki == kj) {
        v = Akk[ki];
    } else {
        Pt<double> a = pts[ki], c = pts[kj];
        double dx = a.x - c.x, dy = a.y - c.y, dz = a.z - c.z;
        double d = sqrt(dx * dx + dy * dy + dz * dz);
        double zp = a.zeta * c.zeta / sqrt(a.zeta * a.zeta + c.zeta * c.zeta);
        v = d == 0.0 ? 1.1283791670955125739 * zp : erf(zp * d) / d;
    }
    blk[ioff[b] + e] = v;
}

// In-place Gauss-Jordan inversion of one SPD block per workgroup (no pivoting needed for SPD);
// a non-positive pivot flags the block as not positive definite.
__global__ __launch_bounds__(256) void k_rbj_invert(const int *__restrict__ off, const long long *__restrict__ ioff,
                                                    double *__restrict__ blk, int *__restrict__ bad) {
    int b = blockIdx.x;
    int l = off[b + 1] - off[b];
    double *A = blk + ioff[b];
    __shared__ double rowk[1024];
    __shared__ double colk[1024];
    __shared__ double piv_s;
    for (int k = 0; k < l; ++k) {
        if (threadIdx.x == 0) {
            piv_s = A[(long long)k * l + k];
            if (!(piv_s > 0.0)) bad[0] = 1;
        }
        __syncthreads();
        double piv = piv_s;
        if (!(piv > 0.0)) return;
        double ip = 1.0 / piv;
        for (int j = threadIdx.x; j < l; j += blockDim.x) {
            rowk[j] = A[(long long)k * l + j] * ip;
            colk[j] = A[(long long)j * l + k];
        }
        __syncthreads();
        // update every element outside row k (rows walked uniformly, columns across lanes)
        for (int i = 0; i < l; ++i) {
            if (i == k) continue;
            const double ci = colk[i];
            double *Ai = A + (long long)i * l;
            for (int j = threadIdx.x; j < l; j += blockDim.x) Ai[j] = (j == k) ? -ci * ip : Ai[j] - ci * rowk[j];
        }
        __syncthreads();
        for (int j = threadIdx.x; j < l; j += blockDim.x) A[(long long)k * l + j] = (j == k) ? ip : rowk[j];
        __syncthreads();
    }
}

// z[perm[o+i]] = sum_j inv[j][i] r[perm[o+j]] (inverse symmetric); per-group partial of r.z
__global__ __launch_bounds__(256) void k_rbj_apply(const int *__restrict__ perm, const int *__restrict__ off,
                                                   const long long *__restrict__ ioff,
                                                   const double *__restrict__ blk, const double *__restrict__ r,
                                                   double *__restrict__ z, double *__restrict__ dp_rz, int tiles) {
    __shared__ double s[256];
    int b = blockIdx.x;
    int o = off[b], l = off[b + 1] - o;
    int i = blockIdx.y * blockDim.x + threadIdx.x;
    double rz = 0.0;
    if (i < l) {
        const double *Ab = blk + ioff[b];
        double acc = 0.0;
        for (int j = 0; j < l; ++j) acc = fma(Ab[(long long)j * l + i], r[perm[o + j]], acc);
        int ki = perm[o + i];
        z[ki] = acc;
        rz = acc * r[ki];
    }
    s[threadIdx.x] = rz;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if (threadIdx.x < q) s[threadIdx.x] += s[threadIdx.x + q];
        __syncthreads();
    }
    if (threadIdx.x == 0) dp_rz[b * tiles + blockIdx.y] = s[0];
}

static void rbj_setup(pcm_ctx *ctx, pcm_mol *mol, int l, unsigned long long seed) {
    if (mol->rbj_valid && mol->rbj_l == l && mol->rbj_seed == seed) return;
    const int M = mol->M;
    std::vector<double> r(3 * (size_t)M), px(M), py(M), pz(M), zeta(M);
    HIP_OK(hipMemcpyAsync(px.data(), mol->px.p, M * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(py.data(), mol->py.p, M * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(pz.data(), mol->pz.p, M * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(zeta.data(), mol->zeta.p, M * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < M; ++k) {
        r[3 * k] = px[k];
        r[3 * k + 1] = py[k];
        r[3 * k + 2] = pz[k];
    }
    mol->h_rbj_perm.assign(M, 0);
    mol->h_rbj_off.assign(M + 1, 0);
    int nb = host_rbj_partition(M, r.data(), zeta.data(), l, seed, mol->h_rbj_perm.data(), mol->h_rbj_off.data());
    if (nb <= 0) throw PcmError{PCM_E_ARG, "randomized block-Jacobi partition failed"};
    mol->h_rbj_off.resize(nb + 1);
    std::vector<long long> ioff(nb + 1, 0);
    int lmax = 0;
    for (int b = 0; b < nb; ++b) {
        int sz = mol->h_rbj_off[b + 1] - mol->h_rbj_off[b];
        ioff[b + 1] = ioff[b] + (long long)sz * sz;
        lmax = std::max(lmax, sz);
    }
    if (lmax > 1024) throw PcmError{PCM_E_ARG, "RBJ block size above 1024 is not supported"};
    mol->rbj_perm.ensure(M);
    mol->rbj_off.ensure(nb + 1);
    mol->rbj_inv_off.ensure(2 * (nb + 1));  // long long stored in int pairs
    mol->rbj_inv.ensure(ioff[nb]);
    HIP_OK(hipMemcpyAsync(mol->rbj_perm.p, mol->h_rbj_perm.data(), M * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(mol->rbj_off.p, mol->h_rbj_off.data(), (nb + 1) * sizeof(int), hipMemcpyHostToDevice,
                          ctx->stream));
    long long *d_ioff = reinterpret_cast<long long *>(mol->rbj_inv_off.p);
    HIP_OK(hipMemcpyAsync(d_ioff, ioff.data(), (nb + 1) * sizeof(long long), hipMemcpyHostToDevice, ctx->stream));
    MatvecWS w = mv_ws(mol);
    dim3 g1(nb, div_up((long long)lmax * lmax, 256));
    k_rbj_fill<<<g1, 256, 0, ctx->stream>>>(w.p64, mol->Akk.p, mol->rbj_perm.p, mol->rbj_off.p, d_ioff,
                                            mol->rbj_inv.p);
    HIP_LAUNCH_OK();
    HIP_OK(hipMemsetAsync(ctx->iscal.p, 0, sizeof(int), ctx->stream));
    {
        ProfScope psi(ctx, "rbj_invert", (double)ioff[nb]);
        k_rbj_invert<<<nb, 256, 0, ctx->stream>>>(mol->rbj_off.p, d_ioff, mol->rbj_inv.p, ctx->iscal.p);
        HIP_LAUNCH_OK();
    }
    int bad = 0;
    HIP_OK(hipMemcpyAsync(&bad, ctx->iscal.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (bad) throw PcmError{PCM_E_NOTPD, "a randomized block-Jacobi block is not positive definite"};
    mol->rbj_l = l;
    mol->rbj_seed = seed;
    mol->rbj_valid = true;
}

static void rbj_apply(pcm_ctx *ctx, pcm_mol *mol, const double *r, double *z, double *dp_rz, int &n_parts) {
    int nb = (int)mol->h_rbj_off.size() - 1;
    int lmax = 0;
    for (int b = 0; b < nb; ++b) lmax = std::max(lmax, mol->h_rbj_off[b + 1] - mol->h_rbj_off[b]);
    int tiles = div_up(lmax, 256);
    dim3 g(nb, tiles);
    ProfScope ps(ctx, "rbj_apply", (double)mol->M * lmax);
    k_rbj_apply<<<g, 256, 0, ctx->stream>>>(mol->rbj_perm.p, mol->rbj_off.p,
                                            reinterpret_cast<const long long *>(mol->rbj_inv_off.p), mol->rbj_inv.p, r,
                                            z, dp_rz, tiles);
    HIP_LAUNCH_OK();
    n_parts = tiles * nb;
}

// ----------------------------------------------------------------------------------------
// one PCG run on A x = b starting from x (in/out); stops on ||r||_2 < tol or max_it
// returns the number of matvecs; *rn_out = final recurrence residual norm
// ----------------------------------------------------------------------------------------
struct CGVecs {
    double *r, *z, *p, *Ap, *y, *dp1, *dp2, *dp3;
};

static CGVecs cg_vecs(pcm_mol *mol) {
    SolverLayout L = solver_layout(mol->M);
    double *b = mol->sv.p;
    return CGVecs{b + L.r, b + L.z, b + L.p, b + L.Ap, b + L.y, b + L.dp1, b + L.dp2, b + L.dp3};
}

static int pcg_run(pcm_ctx *ctx, pcm_mol *mol, const double *b, double *x, bool x_zero, double tol, int max_it,
                   int precond, int mv_prec, double *hist, double *rn_out) {
    const int M = mol->M;
    CGVecs v = cg_vecs(mol);
    const int nbk = div_up(M, 256);
    int n_rz = nbk;
    // initial residual
    if (!x_zero) {
        matvec(ctx, mol, x, v.y, mv_prec, nullptr);
    }
    k_cg_init<<<nbk, 256, 0, ctx->stream>>>(M, b, x_zero ? nullptr : v.y, v.r, v.z, mol->Akk.p, precond, v.dp1, v.dp2);
    HIP_LAUNCH_OK();
    if (precond == PCM_PRECOND_RBJ) rbj_apply(ctx, mol, v.r, v.z, v.dp2, n_rz);
    // hist[0]: rr from dp1 (nbk parts), rz from dp2 (n_rz parts); p = z
    {
        // k_cg_start sums both with the same count; pad when counts differ by summing separately
        k_sum_parts<<<1, 256, 0, ctx->stream>>>(v.dp1, nbk, hist + 2);
        k_sum_parts<<<1, 256, 0, ctx->stream>>>(v.dp2, n_rz, hist + 3);
        k_scale_copy<<<nbk, 256, 0, ctx->stream>>>(M, 1.0, v.z, v.p);
        HIP_LAUNCH_OK();
    }
    double rr = 0.0;
    HIP_OK(hipMemcpyAsync(&rr, hist + 2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    int it = 0;
    double rn = sqrt(rr);
    while (rn >= tol && it < max_it) {
        ++it;
        matvec(ctx, mol, v.p, v.Ap, mv_prec, v.dp3);
        k_cg_update<<<nbk, 256, 0, ctx->stream>>>(M, v.dp3, nbk, hist, it, x, v.r, v.p, v.Ap, v.z, mol->Akk.p,
                                                  precond, v.dp1, v.dp2);
        HIP_LAUNCH_OK();
        if (precond == PCM_PRECOND_RBJ) rbj_apply(ctx, mol, v.r, v.z, v.dp2, n_rz);
        k_cg_direction<<<nbk, 256, 0, ctx->stream>>>(M, v.dp1, nbk, v.dp2, n_rz, hist, it, v.p, v.z);
        HIP_LAUNCH_OK();
        HIP_OK(hipMemcpyAsync(&rr, hist + it * HS + 2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        rn = sqrt(rr);
    }
    *rn_out = rn;
    return it;
}

pcm_status run_solve(pcm_ctx *ctx, pcm_mol *mol, const double *vin, const pcm_solve_opts &o, double *q,
                     pcm_solve_info *info) {
    const int M = mol->M;
    ensure_solver_ws(ctx, mol);
    const double f = (ctx->prm.eps - 1.0) / (ctx->prm.eps + ctx->prm.k_factor);
    SolverLayout SL = solver_layout(M);
    double *b = mol->sv.p + SL.b;      // right-hand side -f v
    double *d = mol->sv.p + SL.d;      // correction (mixed)
    double *res = mol->sv.p + SL.res;  // FP64 residual
    DevBuf<double> &hist = mol->hist;
    hist.ensure((size_t)HS * (o.max_iter + 2) + 16);
    const int nbk = div_up(M, 256);
    auto t0 = std::chrono::steady_clock::now();
    k_scale_copy<<<nbk, 256, 0, ctx->stream>>>(M, -f, vin, b);
    HIP_LAUNCH_OK();
    if (!o.warm_start) HIP_OK(hipMemsetAsync(q, 0, sizeof(double) * M, ctx->stream));
    if (o.precond == PCM_PRECOND_RBJ) rbj_setup(ctx, mol, o.block, o.seed);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    auto t1 = std::chrono::steady_clock::now();
    int iters = 0, refinements = 0;
    double rn = 0.0;
    bool conv = false;
    if (o.precision == PCM_MIXED) {
        // iterative refinement: r = b - A64 q; inner FP32-matvec PCG on A d = r; q += d
        double eta = o.inner_rtol > 0 ? o.inner_rtol : 1e-4;
        while (true) {
            matvec(ctx, mol, q, res, PCM_FP64, nullptr);
            ++iters;
            // res = b - A q
            k_scale_copy<<<nbk, 256, 0, ctx->stream>>>(M, -1.0, res, res);
            k_axpy<<<nbk, 256, 0, ctx->stream>>>(M, 1.0, b, res);
            HIP_LAUNCH_OK();
            double rr = dev_dot(ctx, mol, res, res, M);
            rn = sqrt(rr);
            if (rn < o.tol) {
                conv = true;
                break;
            }
            if (iters >= o.max_iter) break;
            HIP_OK(hipMemsetAsync(d, 0, sizeof(double) * M, ctx->stream));
            double rin = 0.0;
            int left = o.max_iter - iters;
            int n = pcg_run(ctx, mol, res, d, true, std::max(eta * rn, 0.5 * o.tol), left, o.precond, PCM_MIXED,
                            hist.p, &rin);
            iters += n;
            k_axpy<<<nbk, 256, 0, ctx->stream>>>(M, 1.0, d, q);
            HIP_LAUNCH_OK();
            ++refinements;
            if (refinements > 200) break;
        }
    } else {
        double rin = 0.0;
        iters = pcg_run(ctx, mol, b, q, !o.warm_start, o.tol, o.max_iter, o.precond, PCM_FP64, hist.p, &rin);
        // true FP64 residual at exit
        matvec(ctx, mol, q, res, PCM_FP64, nullptr);
        k_scale_copy<<<nbk, 256, 0, ctx->stream>>>(M, -1.0, res, res);
        k_axpy<<<nbk, 256, 0, ctx->stream>>>(M, 1.0, b, res);
        HIP_LAUNCH_OK();
        rn = sqrt(dev_dot(ctx, mol, res, res, M));
        conv = rin < o.tol;
    }
    HIP_OK(hipStreamSynchronize(ctx->stream));
    auto t2 = std::chrono::steady_clock::now();
    if (info) {
        info->iters = iters;
        info->refinements = refinements;
        info->resid = rn;
        // Eq. 13 at q: v.q + 1/(2f) q.Aq with A q = b - res
        double vq = dev_dot(ctx, mol, vin, q, M);
        double bq = dev_dot(ctx, mol, b, q, M);
        double rq = dev_dot(ctx, mol, res, q, M);
        info->energy = vq + 0.5 / f * (bq - rq);
        info->setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->solve_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
    }
    return conv ? PCM_OK : PCM_E_NOCONV;
}

double run_energy(pcm_ctx *ctx, pcm_mol *mol, const double *bz, const double *c, const double *q) {
    ensure_solver_ws(ctx, mol);
    const int M = mol->M;
    const double f = (ctx->prm.eps - 1.0) / (ctx->prm.eps + ctx->prm.k_factor);
    double *Aq = mol->sv.p + solver_layout(M).res;
    matvec(ctx, mol, q, Aq, PCM_FP64, nullptr);
    double e1 = dev_dot(ctx, mol, bz, q, M);
    double e2 = dev_dot(ctx, mol, c, q, M);
    double e3 = dev_dot(ctx, mol, q, Aq, M);
    return e1 + e2 + 0.5 / f * e3;
}

// ----------------------------------------------------------------------------------------
// host partition (Sec. 4b-ii); built with IEEE double and no contraction so that the ranking
// values are the plain expressions erf(z' d)/d, z' = z_k z_l / sqrt(z_k^2 + z_l^2).  For
// z' d >= 6 erf rounds to exactly 1 in double precision, so 1/d is the same value.
// The l-1 best candidates of a pivot are kept in a bounded heap.  Because |A_kl| <= 1/d, a
// candidate farther than 1/(worst kept value) cannot enter and is rejected from its distance
// alone; the ranking is a total order (value, then index), so the selected set is the same as
// a full sort would give.
// ----------------------------------------------------------------------------------------
static inline uint64_t splitmix64_next(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

#pragma clang fp contract(off)
static inline double coupling(const double *r, const double *zeta, int k, int l) {
    double zk = zeta[k], zl = zeta[l];
    double zp = zk * zl / std::sqrt(zk * zk + zl * zl);
    double dx = r[3 * k] - r[3 * l], dy = r[3 * k + 1] - r[3 * l + 1], dz = r[3 * k + 2] - r[3 * l + 2];
    double d = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (d == 0.0) return 2.0 * zp / std::sqrt(M_PI);
    double x = zp * d;
    if (x >= 6.0) return 1.0 / d;
    return std::erf(x) / d;
}

int host_rbj_partition(int M, const double *r, const double *zeta, int l, unsigned long long seed, int *perm,
                       int *blk_off) {
    if (M <= 0 || l <= 0 || !r || !zeta || !perm || !blk_off) return -1;
    // unassigned indices: a Fenwick tree over [0, M) answers "k-th unassigned in ascending
    // order" for the pivot pick; the scan list is compacted lazily
    std::vector<int> bit(M + 1, 0);
    for (int i = 1; i <= M; ++i) {
        bit[i] += 1;
        int j = i + (i & -i);
        if (j <= M) bit[j] += bit[i];
    }
    int top_pow = 1;
    while (top_pow * 2 <= M) top_pow *= 2;
    auto kth = [&](int k) {  // 0-based k-th unassigned index
        int p0 = 0;
        for (int step = top_pow; step > 0; step >>= 1)
            if (p0 + step <= M && bit[p0 + step] <= k) {
                p0 += step;
                k -= bit[p0];
            }
        return p0;  // index (0-based) of the element
    };
    auto remove = [&](int i) {
        for (int j = i + 1; j <= M; j += j & -j) bit[j] -= 1;
    };
    std::vector<int> left(M);
    std::iota(left.begin(), left.end(), 0);
    int n_scan = M;  // entries in left[], some possibly assigned already
    std::vector<unsigned char> take(M, 0);
    using Cand = std::pair<double, int>;
    // heap ordered so that top() is the worst kept candidate (smallest value, then largest index)
    auto better = [](const Cand &a, const Cand &b) {
        return a.first > b.first || (a.first == b.first && a.second < b.second);
    };
    std::vector<Cand> heap;
    heap.reserve(std::min(l, M) + 1);
    uint64_t st = seed;
    int n_left = M, nb = 0, filled = 0;
    blk_off[0] = 0;
    while (n_left > 0) {
        uint64_t x = splitmix64_next(st);
        double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
        int pos = (int)std::floor(u * (double)n_left);
        if (pos >= n_left) pos = n_left - 1;
        const int piv = kth(pos);
        const int want = std::min(l - 1, n_left - 1);
        heap.clear();
        if (want > 0) {
            if (n_scan > 2 * n_left) {  // drop assigned entries before scanning
                int w = 0;
                for (int t = 0; t < n_scan; ++t)
                    if (!take[left[t]]) left[w++] = left[t];
                n_scan = w;
            }
            const double px = r[3 * piv], py = r[3 * piv + 1], pz = r[3 * piv + 2];
            double reject_d2 = 1e300;  // candidates with d^2 above this cannot enter the heap
            for (int t = 0; t < n_scan; ++t) {
                const int q = left[t];
                if (q == piv || take[q]) continue;
                const double dx = px - r[3 * q], dy = py - r[3 * q + 1], dz = pz - r[3 * q + 2];
                const double d2 = dx * dx + dy * dy + dz * dz;
                if ((int)heap.size() == want && d2 > reject_d2) continue;  // |A| <= 1/d < worst kept
                Cand c(std::fabs(coupling(r, zeta, piv, q)), q);
                if ((int)heap.size() < want) {
                    heap.push_back(c);
                    std::push_heap(heap.begin(), heap.end(), better);
                } else if (better(c, heap.front())) {
                    std::pop_heap(heap.begin(), heap.end(), better);
                    heap.back() = c;
                    std::push_heap(heap.begin(), heap.end(), better);
                } else {
                    continue;
                }
                if ((int)heap.size() == want) {
                    const double w = heap.front().first;
                    // |A| <= 1/d: reject when d^2 w^2 > 1 (with a relative margin far above rounding)
                    reject_d2 = w > 0.0 ? (1.0 + 1e-9) / (w * w) : 1e300;
                }
            }
        }
        int start = filled;
        perm[filled++] = piv;
        take[piv] = 1;
        remove(piv);
        for (const Cand &c : heap) {
            perm[filled++] = c.second;
            take[c.second] = 1;
            remove(c.second);
        }
        std::sort(perm + start, perm + filled);
        n_left -= filled - start;
        blk_off[++nb] = filled;
    }
    return nb;
}
