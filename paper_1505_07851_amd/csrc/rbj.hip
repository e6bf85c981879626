// Block-Jacobi preconditioners (Sec. 4b-ii): the randomized partition and the spatial octree
// partition it is compared with (host), and the explicit inverses of the diagonal blocks of
// the permuted A (device).
#include "pcm_internal.h"

#include <algorithm>
#include <cstdlib>
#include <future>
#include <numeric>

// ----------------------------------------------------------------------------------------
// blocks of A gathered by the partition; A_kl from Eqs. 2-3, 8
// ----------------------------------------------------------------------------------------
__global__ void k_rbj_fill(const double *__restrict__ px, const double *__restrict__ py,
                           const double *__restrict__ pz, const double *__restrict__ zeta,
                           const double *__restrict__ Akk, const int *__restrict__ perm, const int *__restrict__ off,
                           const long long *__restrict__ ioff, double *__restrict__ blk) {
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
        double dx = px[ki] - px[kj], dy = py[ki] - py[kj], dz = pz[ki] - pz[kj];
        double d = sqrt(dx * dx + dy * dy + dz * dz);
        double za = zeta[ki], zc = zeta[kj];
        double zp = za * zc / sqrt(za * za + zc * zc);
        v = d == 0.0 ? 1.1283791670955125739 * zp : erf(zp * d) / d;
    }
    blk[ioff[b] + e] = v;
}

// In-place blocked Gauss-Jordan inversion of every SPD block (no pivoting is needed for SPD
// matrices).  Panel K of width GJ_PB is eliminated in four launches over all blocks:
//   diag      A_KK <- P^-1, P = A_KK (scalar Gauss-Jordan, rows in registers; a non-positive pivot flags
//             the block as not positive definite)
//   row       A_Kj <- P^-1 A_Kj                  (j outside K)
//   trailing  A_ij <- A_ij - A_iK A_Kj           (i, j outside K; A_Kj already updated)
//   column    A_iK <- -A_iK P^-1                 (i outside K)
// After the last panel the block holds its inverse.  Each pass over the block is one rank-GJ_PB
// update, so HBM traffic is l^2 per panel instead of per pivot.
constexpr int GJ_PB = 64;
constexpr int GJ_LD = GJ_PB + 1;  // LDS row stride (odd: column walks do not hit one bank)

__device__ inline bool gj_panel(const int *__restrict__ off, const long long *__restrict__ ioff, int b, int p,
                                double *__restrict__ blk, double *&A, int &l, int &K0, int &kb) {
    l = off[b + 1] - off[b];
    K0 = p * GJ_PB;
    if (K0 >= l) return false;
    kb = min(GJ_PB, l - K0);
    A = blk + ioff[b];
    return true;
}

// Diagonal tile: thread (i, q) = (threadIdx.x % 64, threadIdx.x / 64) keeps row i, columns
// 16 q .. 16 q + 15 of the panel in registers, so wave q holds one column quarter of all rows.  Pivot
// step k publishes row k and column k through LDS (double-buffered: one barrier per step), then
// every thread updates its 16 entries with one FMA each:
//   row k:        P_kj <- P_kj / P_kk,            P_kk <- 1 / P_kk
//   other rows i: P_ij <- P_ij - (P_ik / P_kk) P_kj,  P_ik <- -P_ik / P_kk
// A ragged last panel (kb < 64) is padded with the identity, which the steps k < kb leave alone.
__global__ __launch_bounds__(256) void k_gj_diag(const int *__restrict__ off, const long long *__restrict__ ioff,
                                                 double *__restrict__ blk, int p, int *__restrict__ bad) {
    double *A;
    int l, K0, kb;
    if (!gj_panel(off, ioff, blockIdx.x, p, blk, A, l, K0, kb)) return;
    __shared__ double rowb[2][GJ_PB];
    __shared__ double colb[2][GJ_PB];
    const int i = threadIdx.x % GJ_PB, q = threadIdx.x / GJ_PB;
    constexpr int QW = GJ_PB / 4;  // columns per thread
    double v[QW];
#pragma unroll
    for (int c = 0; c < QW; ++c) {
        const int j = QW * q + c;
        v[c] = (i < kb && j < kb) ? A[(long long)(K0 + i) * l + K0 + j] : (i == j ? 1.0 : 0.0);
    }
    for (int kq = 0; kq < 4; ++kq) {  // pivot k = QW kq + kc: kc indexes the registers statically
#pragma unroll
        for (int kc = 0; kc < QW; ++kc) {
            const int k = QW * kq + kc;
            if (k >= kb) break;
            const int bs = kc & 1;
            if (i == k) {
#pragma unroll
                for (int c = 0; c < QW; ++c) rowb[bs][QW * q + c] = v[c];
            }
            if (q == kq) colb[bs][i] = v[kc];
            __syncthreads();
            const double piv = rowb[bs][k];
            if (!(piv > 0.0)) {  // uniform: every thread read the same pivot
                if (threadIdx.x == 0) bad[0] = 1;
                return;
            }
            const double ip = 1.0 / piv;
            const bool rk = i == k;
            const double g = rk ? ip : -(colb[bs][i] * ip);  // the new P_ik
            const double h = rk ? ip - 1.0 : g;              // row k: P_kj + (1/P_kk - 1) P_kj
#pragma unroll
            for (int c = 0; c < QW; ++c) {
                const double nv = fma(h, rowb[bs][QW * q + c], v[c]);
                v[c] = (c == kc && q == kq) ? g : nv;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < QW; ++c) {
        const int j = QW * q + c;
        if (i < kb && j < kb) A[(long long)(K0 + i) * l + K0 + j] = v[c];
    }
}

// Off-diagonal tiles of panel K, one 64 x 64 tile per workgroup:
//   GJ_ROW    tile (K, t):  A_Kt <- P^-1 A_Kt          (P^-1 = the inverted diagonal tile)
//   GJ_TRAIL  tile (s, t):  A_st <- A_st - A_sK A_Kt   (s, t != K; A_Kt already updated)
//   GJ_COL    tile (s, K):  A_sK <- -A_sK P^-1
// Each is out = L R with L[i][m] = A[r0 + i][K0 + m] and R[m][j] = A[K0 + m][c0 + j] for the
// tile's row and column origins (r0, c0), staged in LDS.  A lane accumulates a 4 x 4 sub-tile
// (rows 4 (lane / 16) + u, columns lane % 16 + 16 v), reading 8 LDS values per 16 FMAs.
// Workgroup w serves block 8 (w / (8 T)) + w % 8, tile (w / 8) % T of its T tiles: workgroups
// are dealt to the 8 XCDs in turn, so every tile of a block runs on one XCD and the panel row and
// column it shares are fetched into that XCD's L2 once.
enum { GJ_ROW = 0, GJ_TRAIL = 1, GJ_COL = 2 };
constexpr int GJ_XCD = 8;

__global__ __launch_bounds__(256) void k_gj_update(const int *__restrict__ off, const long long *__restrict__ ioff,
                                                   double *__restrict__ blk, int nb, int p, int nt, int mode) {
    const int T = mode == GJ_TRAIL ? nt * nt : nt;
    const int w = blockIdx.x;
    const int b = GJ_XCD * (w / (GJ_XCD * T)) + w % GJ_XCD, tile = (w / GJ_XCD) % T;
    if (b >= nb) return;
    double *A;
    int l, K0, kb;
    if (!gj_panel(off, ioff, b, p, blk, A, l, K0, kb)) return;
    int ts, tt;  // tile row and column
    if (mode == GJ_TRAIL) {
        ts = tile / nt;
        tt = tile % nt;
        if (ts == p || tt == p) return;
    } else {
        if (tile == p) return;
        ts = mode == GJ_ROW ? p : tile;
        tt = mode == GJ_ROW ? tile : p;
    }
    const int r0 = ts * GJ_PB, c0 = tt * GJ_PB;
    if (r0 >= l || c0 >= l) return;
    const int in = min(GJ_PB, l - r0), jn = min(GJ_PB, l - c0);
    const int u0 = 4 * (threadIdx.x / 16), v0 = threadIdx.x % 16;
    double acc[4][4] = {};
    if (mode == GJ_TRAIL) {  // the old tile, loaded while the panels are staged
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (u0 + u < in && v0 + 16 * v < jn) acc[u][v] = A[(long long)(r0 + u0 + u) * l + c0 + v0 + 16 * v];
    }
    // staging: thread (x, y) = (threadIdx.x % 64, threadIdx.x / 64) loads rows y + 4 s of both
    // panels at column x, all 32 loads in flight before the first LDS store
    __shared__ double Ls[GJ_PB * GJ_LD];  // Ls[m][i] = A[r0 + i][K0 + m] (negated when trailing)
    __shared__ double Rs[GJ_PB * GJ_LD];  // Rs[m][j] = A[K0 + m][c0 + j]
    constexpr int NS = GJ_PB * GJ_PB / 256;
    const int x = threadIdx.x % GJ_PB, y = threadIdx.x / GJ_PB;
    double lv[NS], rv[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int i = y + 4 * t;
        lv[t] = i < in && x < kb ? A[(long long)(r0 + i) * l + K0 + x] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int m = y + 4 * t;
        rv[t] = m < kb && x < jn ? A[(long long)(K0 + m) * l + c0 + x] : 0.0;
    }
    const double sg = mode == GJ_TRAIL ? -1.0 : 1.0;  // trailing: acc = A_st - sum, else sum
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        Ls[x * GJ_LD + y + 4 * t] = sg * lv[t];
        Rs[(y + 4 * t) * GJ_LD + x] = rv[t];
    }
    __syncthreads();
    for (int m = 0; m < kb; ++m) {
        double a[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = Ls[m * GJ_LD + u0 + u];
#pragma unroll
        for (int v = 0; v < 4; ++v) bv[v] = Rs[m * GJ_LD + v0 + 16 * v];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], bv[v], acc[u][v]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = u0 + u;
        if (i >= in) continue;
        double *Ai = A + (long long)(r0 + i) * l + c0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = v0 + 16 * v;
            if (j >= jn) continue;
            Ai[j] = mode == GJ_COL ? -acc[u][v] : acc[u][v];
        }
    }
}

// current kept points (interleaved xyz) and exponents, copied to the host
static void positions_to_host(pcm_ctx *ctx, pcm_mol *mol, std::vector<double> &r, std::vector<double> &zeta) {
    const int M = mol->M;
    std::vector<double> px(M), py(M), pz(M);
    zeta.resize(M);
    r.resize(3 * (size_t)M);
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
}

// The partition depends only on the points, so after a geometry update it is started on a
// host thread for the block size and seed used last; the next solve with the same options
// joins it instead of partitioning while the GPU waits.
struct RbjPending {
    int kind = 0;
    int l = 0;
    unsigned long long seed = 0;
    std::vector<double> r, zeta;
    std::vector<int> perm, off;
    std::future<int> nb;
};

void rbj_pending_drop(pcm_mol *mol) {
    if (!mol->rbj_pending) return;
    if (mol->rbj_pending->nb.valid()) mol->rbj_pending->nb.wait();
    delete mol->rbj_pending;
    mol->rbj_pending = nullptr;
}

void rbj_prefetch(pcm_ctx *ctx, pcm_mol *mol) {
    rbj_pending_drop(mol);
    if (mol->rbj_l < 1 || mol->M < 1) return;  // no block-Jacobi solve on this molecule yet
    RbjPending *p = new RbjPending();
    p->kind = mol->rbj_kind;
    p->l = mol->rbj_l;
    p->seed = mol->rbj_seed;
    try {
        positions_to_host(ctx, mol, p->r, p->zeta);
        const int M = mol->M;
        p->perm.assign(M, 0);
        p->off.assign(M + 1, 0);
        p->nb = std::async(std::launch::async, [p, M]() {
            return block_partition(p->kind, M, p->r.data(), p->zeta.data(), p->l, p->seed, p->perm.data(),
                                   p->off.data());
        });
    } catch (const std::system_error &) {
        delete p;  // no thread available: the solve partitions synchronously
        return;
    } catch (...) {
        delete p;
        throw;
    }
    mol->rbj_pending = p;
}

void rbj_setup(pcm_ctx *ctx, pcm_mol *mol, int kind, int l, unsigned long long seed) {
    if (kind == PCM_PRECOND_OCTREE) seed = 0;  // the octree partition draws no random numbers
    if (mol->rbj_valid && mol->rbj_kind == kind && mol->rbj_l == l && mol->rbj_seed == seed) return;
    const int M = mol->M;
    int nb;
    RbjPending *pd = mol->rbj_pending;
    if (pd && pd->kind == kind && pd->l == l && pd->seed == seed) {
        nb = mol->rbj_pending->nb.get();
        mol->h_rbj_perm = std::move(mol->rbj_pending->perm);
        mol->h_rbj_off = std::move(mol->rbj_pending->off);
        rbj_pending_drop(mol);
    } else {
        rbj_pending_drop(mol);
        std::vector<double> r, zeta;
        positions_to_host(ctx, mol, r, zeta);
        mol->h_rbj_perm.assign(M, 0);
        mol->h_rbj_off.assign(M + 1, 0);
        nb = block_partition(kind, M, r.data(), zeta.data(), l, seed, mol->h_rbj_perm.data(), mol->h_rbj_off.data());
    }
    if (nb <= 0) throw PcmError{PCM_E_ARG, "block-Jacobi partition failed"};
    mol->h_rbj_off.resize(nb + 1);
    std::vector<long long> ioff(nb + 1, 0);
    int lmax = 0;
    for (int b = 0; b < nb; ++b) {
        int sz = mol->h_rbj_off[b + 1] - mol->h_rbj_off[b];
        ioff[b + 1] = ioff[b] + (long long)sz * sz;
        lmax = std::max(lmax, sz);
    }
    if (lmax > 1024) throw PcmError{PCM_E_ARG, "block-Jacobi block size above 1024 is not supported"};
    mol->rbj_lmax = lmax;
    mol->rbj_perm.ensure(M);
    mol->rbj_off.ensure(nb + 1);
    mol->rbj_ioff.ensure(nb + 1);
    mol->rbj_inv.ensure(ioff[nb]);
    HIP_OK(hipMemcpyAsync(mol->rbj_perm.p, mol->h_rbj_perm.data(), M * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(mol->rbj_off.p, mol->h_rbj_off.data(), (nb + 1) * sizeof(int), hipMemcpyHostToDevice,
                          ctx->stream));
    HIP_OK(hipMemcpyAsync(mol->rbj_ioff.p, ioff.data(), (nb + 1) * sizeof(long long), hipMemcpyHostToDevice,
                          ctx->stream));
    dim3 g1(nb, div_up((long long)lmax * lmax, 256));
    k_rbj_fill<<<g1, 256, 0, ctx->stream>>>(mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p, mol->Akk.p,
                                            mol->rbj_perm.p, mol->rbj_off.p, mol->rbj_ioff.p, mol->rbj_inv.p);
    HIP_LAUNCH_OK();
    HIP_OK(hipMemsetAsync(ctx->iscal.p, 0, sizeof(int), ctx->stream));
    {
        ProfScope psi(ctx, "rbj_invert", (double)ioff[nb]);
        const int nt = div_up(lmax, GJ_PB);
        for (int p = 0; p < nt; ++p) {
            k_gj_diag<<<nb, 256, 0, ctx->stream>>>(mol->rbj_off.p, mol->rbj_ioff.p, mol->rbj_inv.p, p, ctx->iscal.p);
            HIP_LAUNCH_OK();
            if (nt == 1) continue;  // a single panel: the block is inverted
            for (int mode : {GJ_ROW, GJ_TRAIL, GJ_COL}) {
                const long long T = mode == GJ_TRAIL ? (long long)nt * nt : nt;
                k_gj_update<<<(unsigned)(div_up(nb, GJ_XCD) * GJ_XCD * T), 256, 0, ctx->stream>>>(
                    mol->rbj_off.p, mol->rbj_ioff.p, mol->rbj_inv.p, nb, p, nt, mode);
                HIP_LAUNCH_OK();
            }
        }
    }
    int bad = 0;
    HIP_OK(hipMemcpyAsync(&bad, ctx->iscal.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (bad) throw PcmError{PCM_E_NOTPD, "a block-Jacobi block is not positive definite"};
    mol->rbj_kind = kind;
    mol->rbj_l = l;
    mol->rbj_seed = seed;
    mol->rbj_valid = true;
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
        return p0;
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

// ----------------------------------------------------------------------------------------
// spatial octree partition (the block-Jacobi scheme RBJ is compared with in Sec. 4b-ii): the
// root is the cube centred on the bounding-box midpoint with half-side half the largest
// extent; a cell with more than leaf_max points is cut into octants at its centre (octant
// bit d set when coordinate d >= centre d), children are visited depth first in octant order,
// empty cells are dropped and a leaf keeps its points in ascending index.  Cells still too
// full at depth 40 (coincident points) are cut into consecutive runs of leaf_max points.
// ----------------------------------------------------------------------------------------
namespace {
constexpr int OCTREE_MAX_DEPTH = 40;

struct OctreeBuild {
    const double *r;
    int leaf_max;
    int *perm, *off;
    int nb = 0, pos = 0;
    std::vector<int> buf;
    std::vector<unsigned char> oct;

    void leaf(const int *p, int n) {
        for (int i = 0; i < n; ++i) perm[pos++] = p[i];
        off[++nb] = pos;
    }
    // p[0, n) is ascending; the stable split keeps every octant ascending
    void visit(int *p, int n, double cx, double cy, double cz, double h, int depth) {
        if (n <= leaf_max) {
            leaf(p, n);
            return;
        }
        if (depth == OCTREE_MAX_DEPTH) {
            for (int s = 0; s < n; s += leaf_max) leaf(p + s, std::min(leaf_max, n - s));
            return;
        }
        int start[9] = {0};
        for (int i = 0; i < n; ++i) {
            const double *x = r + 3 * (size_t)p[i];
            const int o = (x[0] >= cx ? 1 : 0) | (x[1] >= cy ? 2 : 0) | (x[2] >= cz ? 4 : 0);
            oct[i] = (unsigned char)o;
            ++start[o + 1];
        }
        for (int o = 0; o < 8; ++o) start[o + 1] += start[o];
        int fill[8];
        std::copy(start, start + 8, fill);
        for (int i = 0; i < n; ++i) buf[fill[oct[i]]++] = p[i];
        std::copy(buf.begin(), buf.begin() + n, p);
        for (int o = 0; o < 8; ++o) {
            const int cnt = start[o + 1] - start[o];
            if (cnt == 0) continue;
            const double ox = (o & 1) ? 0.5 * h : -0.5 * h, oy = (o & 2) ? 0.5 * h : -0.5 * h,
                         oz = (o & 4) ? 0.5 * h : -0.5 * h;
            visit(p + start[o], cnt, cx + ox, cy + oy, cz + oz, 0.5 * h, depth + 1);
        }
    }
};
}  // namespace

int host_octree_partition(int M, const double *r, int leaf_max, int *perm, int *blk_off) {
    if (M <= 0 || leaf_max <= 0 || !r || !perm || !blk_off) return -1;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = r[d];
    for (int k = 0; k < M; ++k)
        for (int d = 0; d < 3; ++d) {
            const double x = r[3 * (size_t)k + d];
            if (!std::isfinite(x)) return -1;
            lo[d] = std::min(lo[d], x);
            hi[d] = std::max(hi[d], x);
        }
    const double half = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2])) * 0.5;
    std::vector<int> idx(M);
    std::iota(idx.begin(), idx.end(), 0);
    OctreeBuild ob{r, leaf_max, perm, blk_off, 0, 0, {}, {}};
    ob.buf.resize(M);
    ob.oct.resize(M);
    blk_off[0] = 0;
    ob.visit(idx.data(), M, (lo[0] + hi[0]) * 0.5, (lo[1] + hi[1]) * 0.5, (lo[2] + hi[2]) * 0.5, half, 0);
    return ob.nb;
}

int block_partition(int kind, int M, const double *r, const double *zeta, int l, unsigned long long seed, int *perm,
                    int *blk_off) {
    if (kind == PCM_PRECOND_OCTREE) return host_octree_partition(M, r, l, perm, blk_off);
    return host_rbj_partition(M, r, zeta, l, seed, perm, blk_off);
}
