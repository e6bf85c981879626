// Linear solve of Sec. 2, Eq. 1 (A q = -f (Bz + c)) on gfx950, for one molecule or a batch.
//
//  * A x is applied matrix-free (A is never stored): A_kl = erf(zeta'_kl r)/r (Eqs. 2, 8) for
//    k != l, A_kk from Eq. 3.  A is symmetric, so the off-diagonal part is swept over the
//    upper triangle of 256 x 256 point tiles: one workgroup takes the tile pair (I, J), J >= I,
//    one lane per row of I, columns of J wave-uniform.  Each evaluated A_kl feeds the row sum
//    of k and (off-diagonal tiles) the column sum of l, reduced across each 16-lane row by a
//    fixed DPP butterfly and across rows through LDS.
//    Every (tile, row) partial is written to its own slot and the slots are summed in fixed
//    order: results are bitwise reproducible and independent of the launch grid.
//  * erf(zeta' r) rounds to 1 once zeta' r >= 6 (FP64) / 4 (FP32): those pairs take the plain
//    1/r branch, tested with zeta'^2 >= min(zeta_k^2, zeta_l^2)/2.
//  * Preconditioned CG (Sec. 4b) with the residual test ||A q - b||_2 < delta (Eq. 20);
//    Jacobi or randomized block-Jacobi (Sec. 4b-ii) preconditioners.
//  * Mixed precision: FP32 matvec inside FP64 iterative refinement; FP64 vectors, dots and
//    the outer residual.
//  * Batching: every kernel walks a table of work items over a set of molecules; scalars,
//    iteration counters and convergence flags live on the device, per molecule, so groups of
//    iterations run without host round trips and are replayed from a captured hipGraph.
#include "pcm_internal.h"

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <type_traits>

constexpr int TILE = 256;  // points per tile (rows per workgroup)
constexpr int GROUP_K = 8; // PCG iterations per launch group (even: scalar slots alternate)
// Bound on each inner FP32 solve of the refinement: FP32 rounding can stall the inner
// residual above its target on ill-conditioned systems; the outer FP64 residual then restarts.
constexpr int INNER_MAX_IT = 400;
// FP64 solves: restarts from the current q when the recurrence residual converged but the
// recomputed one is not below the threshold
constexpr int MAX_RESTARTS = 3;

template <typename T> struct Pt {
    T x, y, z, zeta;
};

inline int sv_pad(int M) { return (M + TILE - 1) / TILE * TILE; }

// solver vectors of one molecule, each [Mp] with zero tails
enum SolverVec { V_XQ, V_B, V_V, V_RES, V_D, V_R, V_Z, V_P, V_AP, V_Y, V_T, NVEC };

// per-molecule view used by every solver kernel
struct CGMol {
    double *v[NVEC];
    float *p32;               // FP32 copy of the search direction (mixed matvec source)
    const Pt<double> *pt64;   // packed points [Mp]; far dummies past M
    const Pt<float> *pt32;
    const double *Akk;
    double *part;             // [nT][M] matvec partials, slot = the other tile of the pair
    double *dp;               // [3][ndp] reduction partials: 0 p.Ap / residual, 1 r.r, 2 r.z
    const int *perm, *boff;   // RBJ partition (null without RBJ)
    const long long *ioff;
    const double *inv;
    const double *tbox;       // [nT][6] bounding box of each tile's points: min x, y, z, max x, y, z
    const double *boys64;     // Boys tables (near-field A_kl)
    const float *boys32;
    double rc2_64;
    float rc2_32;
    int M, Mp, nT, ndp, n_rz, precond;
};

// per-molecule device state
struct CGState {
    double rz[2];   // r.z of the last two iterations (slot = iteration parity)
    double rr;      // r.r after the last iteration
    double res2;    // ||b - A x||^2 of the last explicit residual
    double tol;     // stop when sqrt(rr) < tol
    double dots[3];
    int it, max_it, done, act;
};

struct MvItem {
    int mol, I, J;
};
struct TileItem {
    int mol, t;
};
struct RbjItem {
    int mol, blk, i0, slot;
};

// ----------------------------------------------------------------------------------------
// device helpers
// ----------------------------------------------------------------------------------------
// A_kl inside the cutoff radius, from the Boys table: erf(z' r)/r = (2/sqrt(pi)) z' F_0(z'^2 r^2)
// (Eq. 3 with F_0(T) = sqrt(pi) erf(sqrt T) / (2 sqrt T)), F_0 by its Taylor series about the
// nearest table node (order 8 in FP64, 4 in FP32; nodes 1/8 apart).  Past z'^2 r^2 = MV_TCUT
// erf has rounded to 1 and A_kl = 1/r = ri.  Coincident points (T = 0) take 2 z'/sqrt(pi).
template <typename T> struct MvCut;
template <> struct MvCut<double> { static constexpr double T_CUT = 36.0; };  // erfc(6) < 3e-17
template <> struct MvCut<float> { static constexpr float T_CUT = 16.0f; };   // erfc(4) < 2e-8
template <typename T>
__device__ __attribute__((noinline)) T mv_near(T zk, T zl, T r2, T ri, bool self, const T *__restrict__ tab) {
    using C = BoysCfg<T>;
    if (self) return T(0);
    const T zp = zk * zl * rsq_fast(fma(zk, zk, zl * zl));
    const T tb = zp * zp * r2;
    if (tb >= MvCut<T>::T_CUT) return ri;
    int i = (int)(tb * T(8) + T(0.5));
    i = i < C::NROW - 1 ? i : C::NROW - 1;
    const T d = T(i) * T(0.125) - tb;
    const T *row = tab + i * C::MT;
    // sum_k F_k(T_i) d^k / k!, nested: F_0 + d (F_1 + d/2 (F_2 + d/3 (...)))
    T F = row[C::ORD];
#pragma unroll
    for (int k = C::ORD; k >= 1; --k) F = fma(F, d * (T(1) / T(k)), row[k - 1]);
    return T(1.1283791670955125739) * zp * F;
}

template <typename T> __device__ __forceinline__ const Pt<T> *mv_pts(const CGMol &m);
template <> __device__ __forceinline__ const Pt<double> *mv_pts<double>(const CGMol &m) { return m.pt64; }
template <> __device__ __forceinline__ const Pt<float> *mv_pts<float>(const CGMol &m) { return m.pt32; }
template <typename T> __device__ __forceinline__ const T *mv_src(const CGMol &m, int src);
template <> __device__ __forceinline__ const double *mv_src<double>(const CGMol &m, int src) { return m.v[src]; }
template <> __device__ __forceinline__ const float *mv_src<float>(const CGMol &m, int) { return m.p32; }
template <typename T> __device__ __forceinline__ T mv_rc2(const CGMol &m);
template <> __device__ __forceinline__ double mv_rc2<double>(const CGMol &m) { return m.rc2_64; }
template <> __device__ __forceinline__ float mv_rc2<float>(const CGMol &m) { return m.rc2_32; }
template <typename T> __device__ __forceinline__ const T *mv_boys(const CGMol &m);
template <> __device__ __forceinline__ const double *mv_boys<double>(const CGMol &m) { return m.boys64; }
template <> __device__ __forceinline__ const float *mv_boys<float>(const CGMol &m) { return m.boys32; }

// gate 0: skip molecules whose PCG is done; gate 1: skip molecules not active in this call
__device__ __forceinline__ bool skip(const CGState &s, int gate) { return gate ? !s.act : s.done; }

// sum over the 256 threads of a block, fixed tree; every thread gets the result
__device__ __forceinline__ double blk_sum(double v, double *s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    double r = s[0];
    __syncthreads();
    return r;
}

// sum of n partials by one block (strided, then the tree)
__device__ __forceinline__ double blk_sum_parts(const double *__restrict__ part, int n, double *s) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    return blk_sum(acc, s);
}

// ----------------------------------------------------------------------------------------
// matrix-free off-diagonal product over the tile pairs of the item table.
// Writes part[J][k] (row sums of tile I against tile J) and, for I != J, part[I][l] (column
// sums of tile J against tile I).  Padded points are far dummies whose x entries are zero.
//
// Lane = 8 i + j.  Wave w owns rows 32 w + 8 a + i (a = 0..3) of tile I, kept in registers with
// their x; tile J's points are staged in LDS and walked in groups of 8 columns (8 b + j).  In a
// group the lane evaluates its 4 pairs (row 8 a + i, column 8 b + j) once: the row terms
// accumulate per a over the whole tile, the column terms per group.  The column sum of a group is
// folded over lane bits 3 (DPP) and 4 (swizzle) and written to LDS per 32-lane half; halves and
// waves are added at the end of the tile.  Row sums are folded over j (lane bits 0-2) by DPP
// once per tile.  Every sum has a fixed order, so results are bitwise reproducible.
// ----------------------------------------------------------------------------------------
constexpr int MV_R = 4;                 // rows per lane (a)
constexpr int MV_WAVES = TILE / (8 * MV_R);  // waves per tile pair: 8 i-lanes x MV_R rows each
constexpr int MV_THREADS = 64 * MV_WAVES;

// lanes l and l ^ 16 exchange values (LDS-free swizzle within 32-lane halves)
__device__ __forceinline__ double swz16(double v) {
    constexpr int XOR16 = (0x10 << 10) | 0x1F;  // bit mode: and 0x1F, or 0, xor 0x10
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), XOR16);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), XOR16);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swz16(float v) {
    constexpr int XOR16 = (0x10 << 10) | 0x1F;
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), XOR16));
}

template <typename T>
__global__ __launch_bounds__(MV_THREADS) void k_mv_sym(const CGMol *__restrict__ tab, const CGState *__restrict__ st,
                                                       const MvItem *__restrict__ items, int n_items, int gate,
                                                       int src) {
    __shared__ T colbuf[2 * MV_WAVES][TILE];  // column sums per (wave, 32-lane half)
    __shared__ Pt<T> cpt[TILE];              // tile J points
    __shared__ T cx[TILE];                   // and their x
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane >> 3, j = lane & 7;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const MvItem w = items[it];
        if (skip(st[w.mol], gate)) continue;
        const CGMol &m = tab[w.mol];
        const Pt<T> *__restrict__ pts = mv_pts<T>(m);
        const T *__restrict__ xv = mv_src<T>(m, src);
        const T rc2 = mv_rc2<T>(m);
        const T *__restrict__ boys = mv_boys<T>(m);
        const int r0 = w.I * TILE + wv * (8 * MV_R) + i, c0 = w.J * TILE;
        const bool diag = w.I == w.J;
        if (threadIdx.x < TILE) {
            cpt[threadIdx.x] = pts[c0 + threadIdx.x];
            cx[threadIdx.x] = xv[c0 + threadIdx.x];
        }
        Pt<T> rp[MV_R];
        T rx[MV_R], racc[MV_R];
#pragma unroll
        for (int a = 0; a < MV_R; ++a) {
            rp[a] = pts[r0 + 8 * a];
            rx[a] = xv[r0 + 8 * a];
            racc[a] = T(0);
        }
        __syncthreads();
        // A tile pair whose boxes are farther apart than the cutoff has no near pair: its loop
        // skips the per-pair test.  The diagonal pair (self term, padding dummies) always tests.
        // FP32 keeps the single tested loop: a second copy costs it a wave per SIMD.
        bool near_item = diag || sizeof(T) == 4;
        if (!near_item) {
            const double *bi = m.tbox + 6 * w.I, *bj = m.tbox + 6 * w.J;
            double g2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double g = fmax(fmax(bj[c] - bi[c + 3], bi[c] - bj[c + 3]), 0.0);
                g2 = fma(g, g, g2);
            }
            near_item = g2 < 1.01 * (double)rc2 + 1e-3;
        }
        auto jloop = [&](auto near_c) {
            constexpr bool NEAR = decltype(near_c)::value;
            for (int b = 0; b < TILE / 8; ++b) {
                const int cl = 8 * b + j;
                const Pt<T> cp = cpt[cl];
                const T xc = cx[cl];
                T cacc = T(0);
#pragma unroll
                for (int a = 0; a < MV_R; ++a) {
                    const T dx = rp[a].x - cp.x, dy = rp[a].y - cp.y, dz = rp[a].z - cp.z;
                    const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    T A = rsq_fast(r2);
                    if constexpr (NEAR) {
                        if (r2 < rc2)
                            A = mv_near<T>(rp[a].zeta, cp.zeta, r2, A, diag && r0 + 8 * a == c0 + cl, boys);
                    }
                    racc[a] = fma(A, xc, racc[a]);
                    cacc = fma(A, rx[a], cacc);
                }
                if (!diag) {
                    cacc += dpp<DPP_ROW_ROR8>(cacc);  // i bit 0 (lane bit 3)
                    cacc += swz16(cacc);               // i bit 1 (lane bit 4)
                    if ((lane & 24) == 0) colbuf[wv * 2 + (lane >> 5)][cl] = cacc;
                }
            }
        };
        if constexpr (sizeof(T) == 4) {
            jloop(std::true_type{});
        } else {
            if (__builtin_amdgcn_readfirstlane((int)near_item))
                jloop(std::true_type{});
            else
                jloop(std::false_type{});
        }
        // row sums over j (lane bits 0-2): quad pairs, quads, half rows
#pragma unroll
        for (int a = 0; a < MV_R; ++a) {
            T v = racc[a];
            v += dpp<DPP_QUAD_XOR1>(v);
            v += dpp<DPP_QUAD_XOR2>(v);
            v += dpp<DPP_ROW_HALF_MIRROR>(v);
            const int k = r0 + 8 * a;
            if (j == 0 && k < m.M) m.part[(size_t)w.J * m.M + k] = (double)v;
        }
        __syncthreads();
        if (!diag && threadIdx.x < TILE) {
            const int c = c0 + threadIdx.x;
            T s = colbuf[0][threadIdx.x];
#pragma unroll
            for (int q = 1; q < 2 * MV_WAVES; ++q) s += colbuf[q][threadIdx.x];
            if (c < m.M) m.part[(size_t)w.I * m.M + c] = (double)s;
        }
        __syncthreads();
    }
}

// y = Akk x + sum of the nT partial slots (fixed order).
//   mode 0: v[dst] = y, dp[0] <- partials of x.y
//   mode 1: v[dst] = v[bvec] - y, dp[0] <- partials of its square
//   mode 2: v[dst] = y
// Each row's nT partial slots are summed by FIN_G thread groups (slots r = g mod FIN_G), then
// added in group order: four times the waves of one thread per row hide the load latency.
constexpr int FIN_G = 4;
__global__ __launch_bounds__(TILE * FIN_G) void k_mv_finish(const CGMol *__restrict__ tab,
                                                            const CGState *__restrict__ st,
                                                            const TileItem *__restrict__ items, int n, int gate,
                                                            int src, int dst, int bvec, int mode) {
    __shared__ double s[TILE * FIN_G];
    const int row = threadIdx.x % TILE, g = threadIdx.x / TILE;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const TileItem w = items[it];
        if (skip(st[w.mol], gate)) continue;
        const CGMol &m = tab[w.mol];
        const int k = w.t * TILE + row;
        double off = 0.0;
        if (k < m.M)
            for (int r = g; r < m.nT; r += FIN_G) off += m.part[(size_t)r * m.M + k];
        s[threadIdx.x] = off;
        __syncthreads();
        double d = 0.0;
        if (g == 0 && k < m.M) {
            double o = s[row];
#pragma unroll
            for (int q = 1; q < FIN_G; ++q) o += s[q * TILE + row];
            const double xk = m.v[src][k];
            const double acc = m.Akk[k] * xk + o;
            if (mode == 1) {
                double res = m.v[bvec][k] - acc;
                m.v[dst][k] = res;
                d = res * res;
            } else {
                m.v[dst][k] = acc;
                d = xk * acc;
            }
        }
        __syncthreads();  // s is reused by the block sum
        if (mode != 2) {
            double t = blk_sum(d, s);  // over the first TILE threads; the other groups hold 0
            if (threadIdx.x == 0) m.dp[w.t] = t;
        }
    }
}

// ----------------------------------------------------------------------------------------
// PCG kernels.  x = v[xi], b = v[bi].
// ----------------------------------------------------------------------------------------
// r = b - (zero_x ? 0 : v[V_Y]); x = 0 when zero_x; z = C r (Jacobi / none); partials r.r, r.z
__global__ __launch_bounds__(TILE) void k_cg_init(const CGMol *__restrict__ tab, const CGState *__restrict__ st,
                                                  const TileItem *__restrict__ items, int n, int xi, int bi,
                                                  int zero_x) {
    __shared__ double s[TILE];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const TileItem w = items[it];
        if (st[w.mol].done) continue;
        const CGMol &m = tab[w.mol];
        const int k = w.t * TILE + threadIdx.x;
        double rr = 0.0, rz = 0.0;
        if (k < m.M) {
            double rk = m.v[bi][k] - (zero_x ? 0.0 : m.v[V_Y][k]);
            if (zero_x) m.v[xi][k] = 0.0;
            m.v[V_R][k] = rk;
            rr = rk * rk;
            if (m.precond != PCM_PRECOND_RBJ) {
                double zk = m.precond == PCM_PRECOND_JACOBI ? rk / m.Akk[k] : rk;
                m.v[V_Z][k] = zk;
                rz = rk * zk;
            }
        }
        double a = blk_sum(rr, s);
        if (threadIdx.x == 0) m.dp[m.ndp + w.t] = a;
        if (m.precond != PCM_PRECOND_RBJ) {
            double b = blk_sum(rz, s);
            if (threadIdx.x == 0) m.dp[2 * m.ndp + w.t] = b;
        }
    }
}

// alpha = r.z / p.Ap; x += alpha p; r -= alpha Ap; z = C r (Jacobi / none); partials r.r, r.z
__global__ __launch_bounds__(TILE) void k_cg_update(const CGMol *__restrict__ tab, const CGState *__restrict__ st,
                                                    const TileItem *__restrict__ items, int n, int xi, int par_prev) {
    __shared__ double s[TILE];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const TileItem w = items[it];
        const CGState &S = st[w.mol];
        if (S.done) continue;
        const CGMol &m = tab[w.mol];
        const double pAp = blk_sum_parts(m.dp, m.nT, s);
        const double alpha = S.rz[par_prev] / pAp;
        const int k = w.t * TILE + threadIdx.x;
        double rr = 0.0, rz = 0.0;
        if (k < m.M) {
            m.v[xi][k] += alpha * m.v[V_P][k];
            double rk = m.v[V_R][k] - alpha * m.v[V_AP][k];
            m.v[V_R][k] = rk;
            rr = rk * rk;
            if (m.precond != PCM_PRECOND_RBJ) {
                double zk = m.precond == PCM_PRECOND_JACOBI ? rk / m.Akk[k] : rk;
                m.v[V_Z][k] = zk;
                rz = rk * zk;
            }
        }
        double a = blk_sum(rr, s);
        if (threadIdx.x == 0) m.dp[m.ndp + w.t] = a;
        if (m.precond != PCM_PRECOND_RBJ) {
            double b = blk_sum(rz, s);
            if (threadIdx.x == 0) m.dp[2 * m.ndp + w.t] = b;
        }
    }
}

// randomized block-Jacobi: z[perm[o+i]] = sum_j inv[j][i] r[perm[o+j]] (inverse symmetric);
// partials of r.z per item.  An item is a slab of RBJ_ROWS rows of one block, one row per lane;
// the block's columns are split into TILE / RBJ_ROWS contiguous chunks, one per wave, so a block
// of l points streams its l^2 inverse entries through l / 16 waves.  Each lane has a column
// element of RBJ_UNROLL inverse rows in flight per step (each wave load a 512-byte row segment);
// the chunk sums are added in wave order, so the result is bitwise reproducible.
constexpr int RBJ_ROWS = 64;
constexpr int RBJ_UNROLL = 16;
constexpr int RBJ_SPLIT = TILE / RBJ_ROWS;
__global__ __launch_bounds__(TILE) void k_rbj_items(const CGMol *__restrict__ tab, const CGState *__restrict__ st,
                                                    const RbjItem *__restrict__ items, int n) {
    __shared__ double rb[1024];  // the block's residual entries, gathered once (l <= 1024)
    __shared__ double red[RBJ_SPLIT - 1][RBJ_ROWS];
    const int lane = threadIdx.x % RBJ_ROWS, wv = threadIdx.x / RBJ_ROWS;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const RbjItem w = items[it];
        if (st[w.mol].done) continue;
        const CGMol &m = tab[w.mol];
        const int o = m.boff[w.blk], l = m.boff[w.blk + 1] - o;
        const double *__restrict__ r = m.v[V_R];
        const int *__restrict__ pm = m.perm + o;
        for (int j = threadIdx.x; j < l; j += TILE) rb[j] = r[pm[j]];
        __syncthreads();
        const int i = w.i0 + lane;
        const int cl = (l + RBJ_SPLIT - 1) / RBJ_SPLIT;
        const int j1 = min(l, (wv + 1) * cl);
        double acc = 0.0;
        if (i < l) {
            const double *__restrict__ Ab = m.inv + m.ioff[w.blk] + i;
            for (int j = wv * cl; j < j1; j += RBJ_UNROLL) {
                double a[RBJ_UNROLL];
#pragma unroll
                for (int u = 0; u < RBJ_UNROLL; ++u) a[u] = j + u < j1 ? Ab[(long long)(j + u) * l] : 0.0;
#pragma unroll
                for (int u = 0; u < RBJ_UNROLL; ++u)
                    if (j + u < j1) acc = fma(a[u], rb[j + u], acc);
            }
        }
        if (wv > 0) red[wv - 1][lane] = acc;
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int u = 0; u < RBJ_SPLIT - 1; ++u) acc += red[u][lane];
            double rz = 0.0;
            if (i < l) {
                m.v[V_Z][pm[i]] = acc;
                rz = acc * rb[i];
            }
            for (int d = RBJ_ROWS / 2; d > 0; d >>= 1) rz += __shfl_xor(rz, d, RBJ_ROWS);
            if (lane == 0) m.dp[2 * m.ndp + w.slot] = rz;
        }
        __syncthreads();  // rb and red are rewritten by the next item
    }
}

// beta = r.z / r.z_prev (0 on the first call); p = z + beta p (p = z first); optional FP32
// copy of p.  The block of tile 0 records r.r, r.z, the iteration count and the stop flag.
__global__ __launch_bounds__(TILE) void k_cg_dir(const CGMol *__restrict__ tab, CGState *__restrict__ st,
                                                 const TileItem *__restrict__ items, int n, int par, int first,
                                                 int w32) {
    __shared__ double s[TILE];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const TileItem w = items[it];
        CGState *S = st + w.mol;
        if (S->done) continue;
        const CGMol &m = tab[w.mol];
        const double rr = blk_sum_parts(m.dp + m.ndp, m.nT, s);
        const double rz = blk_sum_parts(m.dp + 2 * m.ndp, m.n_rz, s);
        const double beta = first ? 0.0 : rz / S->rz[par ^ 1];
        const int k = w.t * TILE + threadIdx.x;
        if (k < m.M) {
            const double zk = m.v[V_Z][k];
            const double pk = first ? zk : zk + beta * m.v[V_P][k];
            m.v[V_P][k] = pk;
            if (w32) m.p32[k] = (float)pk;
        }
        if (w.t == 0 && threadIdx.x == 0) {
            S->rz[par] = rz;
            S->rr = rr;
            const int itn = first ? 0 : S->it + 1;
            S->it = itn;
            S->done = (!(sqrt(rr) >= S->tol) || itn >= S->max_it) ? 1 : 0;
        }
    }
}

__global__ __launch_bounds__(TILE) void k_count_active(const CGState *__restrict__ st, int n, int *__restrict__ out) {
    __shared__ double s[TILE];
    double c = 0.0;
    for (int i = threadIdx.x; i < n; i += TILE) c += st[i].done ? 0.0 : 1.0;
    double t = blk_sum(c, s);
    if (threadIdx.x == 0) out[0] = (int)t;
}

// ----------------------------------------------------------------------------------------
// vector plumbing over the tile table (gate 1: molecules with act set)
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_vec_op(const CGMol *__restrict__ tab, const CGState *__restrict__ st,
                                                 const TileItem *__restrict__ items, int n, int op, double a, int src,
                                                 int dst, const double *const *__restrict__ ext) {
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const TileItem w = items[it];
        if (!st[w.mol].act) continue;
        const CGMol &m = tab[w.mol];
        const int k = w.t * TILE + threadIdx.x;
        if (k >= m.M) continue;
        switch (op) {
        case 0: m.v[dst][k] = ext[w.mol][k]; break;                       // load caller vector
        case 1: const_cast<double *>(ext[w.mol])[k] = m.v[src][k]; break;  // store to caller
        case 2: m.v[dst][k] = a * m.v[src][k]; break;                     // scale
        case 3: m.v[dst][k] += a * m.v[src][k]; break;                    // axpy
        case 5: m.v[dst][k] += ext[w.mol][k]; break;                      // add caller vector
        default: m.v[dst][k] = 0.0; break;                                // zero
        }
    }
}

// partials of three dot products v[a_j].v[b_j] into dp[j]
__global__ __launch_bounds__(TILE) void k_dots3(const CGMol *__restrict__ tab, const CGState *__restrict__ st,
                                                const TileItem *__restrict__ items, int n, int a0, int b0, int a1,
                                                int b1, int a2, int b2) {
    __shared__ double s[TILE];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const TileItem w = items[it];
        if (!st[w.mol].act) continue;
        const CGMol &m = tab[w.mol];
        const int k = w.t * TILE + threadIdx.x;
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        if (k < m.M) {
            d0 = m.v[a0][k] * m.v[b0][k];
            d1 = m.v[a1][k] * m.v[b1][k];
            d2 = m.v[a2][k] * m.v[b2][k];
        }
        double t0 = blk_sum(d0, s), t1 = blk_sum(d1, s), t2 = blk_sum(d2, s);
        if (threadIdx.x == 0) {
            m.dp[w.t] = t0;
            m.dp[m.ndp + w.t] = t1;
            m.dp[2 * m.ndp + w.t] = t2;
        }
    }
}

// one block per molecule: what = 0: res2 <- sum dp[0]; what = 1: dots[j] <- sum dp[j]
__global__ __launch_bounds__(TILE) void k_mol_reduce(const CGMol *__restrict__ tab, CGState *__restrict__ st,
                                                     int what) {
    __shared__ double s[TILE];
    CGState *S = st + blockIdx.x;
    if (!S->act) return;
    const CGMol &m = tab[blockIdx.x];
    if (what == 0) {
        double t = blk_sum_parts(m.dp, m.nT, s);
        if (threadIdx.x == 0) S->res2 = t;
    } else {
        for (int j = 0; j < 3; ++j) {
            double t = blk_sum_parts(m.dp + j * m.ndp, m.nT, s);
            if (threadIdx.x == 0) S->dots[j] = t;
        }
    }
}

__global__ void k_pack_pts(const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ pz,
                           const double *__restrict__ zeta, int M, int Mp, Pt<double> *__restrict__ p64,
                           Pt<float> *__restrict__ p32) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mp) return;
    if (k < M) {
        p64[k] = Pt<double>{px[k], py[k], pz[k], zeta[k]};
        p32[k] = Pt<float>{(float)px[k], (float)py[k], (float)pz[k], (float)zeta[k]};
    } else {
        p64[k] = Pt<double>{1e6, 1e6, 1e6, 1.0};
        p32[k] = Pt<float>{1e6f, 1e6f, 1e6f, 1.0f};
    }
}

// bounding box of each tile's real points (block = tile); an empty tail tile gets an empty box
__global__ __launch_bounds__(TILE) void k_tile_box(const Pt<double> *__restrict__ p64, int M, double *__restrict__ tbox) {
    __shared__ double red[6][TILE];
    const int k = blockIdx.x * TILE + threadIdx.x;
    const bool in = k < M;
    const Pt<double> p = p64[in ? k : 0];
    red[0][threadIdx.x] = in ? p.x : 1e300;
    red[1][threadIdx.x] = in ? p.y : 1e300;
    red[2][threadIdx.x] = in ? p.z : 1e300;
    red[3][threadIdx.x] = in ? p.x : -1e300;
    red[4][threadIdx.x] = in ? p.y : -1e300;
    red[5][threadIdx.x] = in ? p.z : -1e300;
    __syncthreads();
    for (int o = TILE / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + o]);
                red[c + 3][threadIdx.x] = fmax(red[c + 3][threadIdx.x], red[c + 3][threadIdx.x + o]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) tbox[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// ----------------------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------------------
// per-molecule solver storage inside mol->sv (offsets in doubles)
struct SvLayout {
    size_t vec[NVEC], p32, pt64, pt32, tbox, total;
};

static SvLayout sv_layout(int M) {
    SvLayout L{};
    const size_t Mp = sv_pad(M);
    size_t o = 0;
    for (int i = 0; i < NVEC; ++i, o += Mp) L.vec[i] = o;
    L.p32 = o;
    o += Mp / 2;
    L.pt64 = o;
    o += 4 * Mp;
    L.pt32 = o;
    o += 2 * Mp;
    L.tbox = o;
    o += 6 * (Mp / TILE);
    L.total = o;
    return L;
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

// allocate (once; zero tails) and pack the current points
static void solver_prepare(pcm_ctx *ctx, pcm_mol *mol) {
    const SvLayout L = sv_layout(mol->M);
    if (mol->sv.n < L.total || !mol->sv.p) {
        mol->sv.ensure(L.total);
        HIP_OK(hipMemsetAsync(mol->sv.p, 0, L.total * sizeof(double), ctx->stream));
    }
    const int Mp = sv_pad(mol->M);
    k_pack_pts<<<grid_for(Mp, 256), 256, 0, ctx->stream>>>(
        mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p, mol->M, Mp,
        reinterpret_cast<Pt<double> *>(mol->sv.p + L.pt64), reinterpret_cast<Pt<float> *>(mol->sv.p + L.pt32));
    HIP_LAUNCH_OK();
    if (Mp > 0) {
        k_tile_box<<<Mp / TILE, TILE, 0, ctx->stream>>>(reinterpret_cast<const Pt<double> *>(mol->sv.p + L.pt64),
                                                        mol->M, mol->sv.p + L.tbox);
        HIP_LAUNCH_OK();
    }
}

struct GraphSig {
    const void *tab, *st, *mv, *tiles, *rbj;
    int n_mv, n_tiles, n_rbj, grid, rbj_on, prec;
    bool operator==(const GraphSig &o) const {
        return tab == o.tab && st == o.st && mv == o.mv && tiles == o.tiles && rbj == o.rbj && n_mv == o.n_mv &&
               n_tiles == o.n_tiles && n_rbj == o.n_rbj && grid == o.grid && rbj_on == o.rbj_on && prec == o.prec;
    }
};

struct SolveBatch {
    std::vector<pcm_mol *> mols;
    int n = 0;
    DevBuf<CGMol> tab;
    DevBuf<CGState> st;
    DevBuf<MvItem> mv;
    DevBuf<TileItem> tiles;
    DevBuf<RbjItem> rbj;
    DevBuf<MvItem> share;  // tile pairs of one rank's share of the product
    DevBuf<double> part, dp;
    DevBuf<const double *> ext;
    DevBuf<int> cnt;
    int n_mv = 0, n_tiles = 0, n_rbj = 0;
    std::vector<CGMol> h_tab;
    std::vector<CGState> h_st;
    std::vector<size_t> part_off, dp_off;
    int *h_cnt = nullptr;  // pinned [2]
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    GraphSig gsig[2] = {};
    ~SolveBatch() {
        for (auto &g : gexec)
            if (g) (void)hipGraphExecDestroy(g);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
        if (h_cnt) (void)hipHostFree(h_cnt);
    }
};

void solve_batch_free(SolveBatch *b) { delete b; }

SolveBatch *solve_batch_new(const std::vector<pcm_mol *> &mols) {
    SolveBatch *b = new SolveBatch();
    b->mols = mols;
    b->n = (int)mols.size();
    return b;
}

static int grid_of(int n) { return n < 1 ? 1 : n; }

// tables that depend on sizes and the RBJ partition; per-call pointers are refreshed each run
static void batch_tables(pcm_ctx *ctx, SolveBatch &B, int precond) {
    // the octree differs from RBJ only in its partition; both apply explicit block inverses
    if (precond == PCM_PRECOND_OCTREE) precond = PCM_PRECOND_RBJ;
    const int n = B.n;
    std::vector<MvItem> mv;
    std::vector<TileItem> tl;
    std::vector<RbjItem> rb;
    B.part_off.assign(n + 1, 0);
    B.dp_off.assign(n + 1, 0);
    B.h_tab.assign(n, CGMol{});
    for (int i = 0; i < n; ++i) {
        pcm_mol *mol = B.mols[i];
        const int M = mol->M, Mp = sv_pad(M), nT = Mp / TILE;
        for (int I = 0; I < nT; ++I)
            for (int J = I; J < nT; ++J) mv.push_back(MvItem{i, I, J});
        for (int t = 0; t < nT; ++t) tl.push_back(TileItem{i, t});
        int n_rz = nT;
        if (precond == PCM_PRECOND_RBJ) {
            const int nb = (int)mol->h_rbj_off.size() - 1;
            int slot = 0;
            for (int bk = 0; bk < nb; ++bk) {
                const int l = mol->h_rbj_off[bk + 1] - mol->h_rbj_off[bk];
                for (int i0 = 0; i0 < l; i0 += RBJ_ROWS) rb.push_back(RbjItem{i, bk, i0, slot++});
            }
            n_rz = slot;
        }
        CGMol &m = B.h_tab[i];
        m.M = M;
        m.Mp = Mp;
        m.nT = nT;
        m.n_rz = n_rz;
        m.ndp = std::max(nT, n_rz);
        m.precond = precond;
        B.part_off[i + 1] = B.part_off[i] + (size_t)nT * M;
        B.dp_off[i + 1] = B.dp_off[i] + 3 * (size_t)m.ndp;
    }
    B.n_mv = (int)mv.size();
    B.n_tiles = (int)tl.size();
    B.n_rbj = (int)rb.size();
    B.tab.ensure(n);
    B.st.ensure(n);
    B.ext.ensure(n);
    B.cnt.ensure(2);
    B.mv.ensure(std::max<size_t>(mv.size(), 1));
    B.tiles.ensure(std::max<size_t>(tl.size(), 1));
    B.rbj.ensure(std::max<size_t>(rb.size(), 1));
    B.part.ensure(std::max<size_t>(B.part_off[n], 1));
    B.dp.ensure(std::max<size_t>(B.dp_off[n], 1));
    HIP_OK(hipMemcpyAsync(B.mv.p, mv.data(), mv.size() * sizeof(MvItem), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(B.tiles.p, tl.data(), tl.size() * sizeof(TileItem), hipMemcpyHostToDevice, ctx->stream));
    if (!rb.empty())
        HIP_OK(hipMemcpyAsync(B.rbj.p, rb.data(), rb.size() * sizeof(RbjItem), hipMemcpyHostToDevice, ctx->stream));
    for (int i = 0; i < n; ++i) {
        pcm_mol *mol = B.mols[i];
        CGMol &m = B.h_tab[i];
        const SvLayout L = sv_layout(mol->M);
        for (int v = 0; v < NVEC; ++v) m.v[v] = mol->sv.p + L.vec[v];
        m.p32 = reinterpret_cast<float *>(mol->sv.p + L.p32);
        m.pt64 = reinterpret_cast<const Pt<double> *>(mol->sv.p + L.pt64);
        m.pt32 = reinterpret_cast<const Pt<float> *>(mol->sv.p + L.pt32);
        m.tbox = mol->sv.p + L.tbox;
        m.Akk = mol->Akk.p;
        m.part = B.part.p + B.part_off[i];
        m.dp = B.dp.p + B.dp_off[i];
        if (precond == PCM_PRECOND_RBJ) {
            m.perm = mol->rbj_perm.p;
            m.boff = mol->rbj_off.p;
            m.ioff = mol->rbj_ioff.p;
            m.inv = mol->rbj_inv.p;
        }
        if (!ctx->boys64.p || !ctx->boys32.p) throw PcmError{PCM_E_STATE, "Boys tables not initialised"};
        m.boys64 = ctx->boys64.p;
        m.boys32 = ctx->boys32.p;
        double r32;
        mv_cutoffs(mol, m.rc2_64, r32);
        m.rc2_32 = (float)r32;
    }
    HIP_OK(hipMemcpyAsync(B.tab.p, B.h_tab.data(), n * sizeof(CGMol), hipMemcpyHostToDevice, ctx->stream));
    if (!B.h_cnt) HIP_OK(hipHostMalloc((void **)&B.h_cnt, 2 * sizeof(int), hipHostMallocDefault));
    for (auto &e : B.ev)
        if (!e) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

static void upload_states(pcm_ctx *ctx, SolveBatch &B) {
    // a molecule without surface points has nothing to iterate (its tile kernels never run,
    // so the device would never set its stop flag)
    for (int i = 0; i < B.n; ++i)
        if (B.h_tab[i].M == 0) B.h_st[i].done = 1;
    HIP_OK(hipMemcpyAsync(B.st.p, B.h_st.data(), B.n * sizeof(CGState), hipMemcpyHostToDevice, ctx->stream));
}

static void download_states(pcm_ctx *ctx, SolveBatch &B) {
    HIP_OK(hipMemcpyAsync(B.h_st.data(), B.st.p, B.n * sizeof(CGState), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
}

// Work of one launch for per-kernel profiling, counted over the molecules that take part
// (host copy of the states, kept current while profiling): unordered point pairs for the
// matvec, inverse-block elements for the RBJ apply.
static bool takes_part(const CGState &h, int gate) { return gate ? h.act != 0 : h.done == 0; }

static double mv_work(const SolveBatch &B, int gate) {
    double w = 0.0;
    for (int i = 0; i < B.n; ++i)
        if (takes_part(B.h_st[i], gate)) w += 0.5 * (double)B.h_tab[i].M * (double)(B.h_tab[i].M - 1);
    return w;
}

static double rbj_work(const SolveBatch &B) {
    double w = 0.0;
    for (int i = 0; i < B.n; ++i) {
        if (!takes_part(B.h_st[i], 0)) continue;
        const std::vector<int> &off = B.mols[i]->h_rbj_off;
        for (size_t b = 0; b + 1 < off.size(); ++b) w += (double)(off[b + 1] - off[b]) * (off[b + 1] - off[b]);
    }
    return w;
}

// ---------------------------------------------------------------- launch grid of the matvec
// The autotuner times the persistent matvec at a few grid sizes on first use for a given
// (precision, item count) and caches the fastest.  The grid does not change any result.
static std::map<std::pair<int, int>, int> g_mv_grid;

static void launch_mv(pcm_ctx *ctx, SolveBatch &B, hipStream_t s, int prec, int gate, int src, int grid) {
    if (prec == PCM_MIXED)
        k_mv_sym<float><<<grid, MV_THREADS, 0, s>>>(B.tab.p, B.st.p, B.mv.p, B.n_mv, gate, src);
    else
        k_mv_sym<double><<<grid, MV_THREADS, 0, s>>>(B.tab.p, B.st.p, B.mv.p, B.n_mv, gate, src);
    HIP_LAUNCH_OK();
}

static int mv_grid(pcm_ctx *ctx, SolveBatch &B, int prec, int gate, int src) {
    if (B.n_mv == 0) return 1;  // every molecule of the batch is empty
    auto key = std::make_pair(prec, B.n_mv);
    auto f = g_mv_grid.find(key);
    if (f != g_mv_grid.end()) return f->second;
    std::vector<int> cand{B.n_mv};
    for (int c : {512, 1024, 2048, 4096, 8192})
        if (c < B.n_mv) cand.push_back(c);
    int best = B.n_mv;
    if (cand.size() > 1) {
        hipEvent_t a, b;
        HIP_OK(hipEventCreate(&a));
        HIP_OK(hipEventCreate(&b));
        float best_ms = 1e30f;
        for (int g : cand) {
            launch_mv(ctx, B, ctx->stream, prec, gate, src, g);
            HIP_OK(hipEventRecord(a, ctx->stream));
            for (int r = 0; r < 3; ++r) launch_mv(ctx, B, ctx->stream, prec, gate, src, g);
            HIP_OK(hipEventRecord(b, ctx->stream));
            HIP_OK(hipEventSynchronize(b));
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, a, b));
            if (ms < best_ms * 0.98f) {
                best_ms = ms;
                best = g;
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    g_mv_grid[key] = best;
    return best;
}

// one matvec: part <- off-diagonal partials of v[src]; then the finish kernel
static void matvec(pcm_ctx *ctx, SolveBatch &B, hipStream_t s, int prec, int gate, int src, int dst, int bvec,
                   int mode, int grid, bool prof) {
    {
        ProfScope ps(prof ? ctx : nullptr, prec == PCM_MIXED ? "matvec_f32" : "matvec_f64",
                     prof ? mv_work(B, gate) : 0.0);
        launch_mv(ctx, B, s, prec, gate, src, grid);
    }
    k_mv_finish<<<grid_of(B.n_tiles), TILE * FIN_G, 0, s>>>(B.tab.p, B.st.p, B.tiles.p, B.n_tiles, gate, src, dst, bvec,
                                                    mode);
    HIP_LAUNCH_OK();
}

// one PCG iteration for every molecule still running; par = iteration parity
static void pcg_iteration(pcm_ctx *ctx, SolveBatch &B, hipStream_t s, int prec, int xi, int par, int grid,
                          bool rbj, bool prof) {
    matvec(ctx, B, s, prec, 0, V_P, V_AP, 0, 0, grid, prof);
    k_cg_update<<<grid_of(B.n_tiles), TILE, 0, s>>>(B.tab.p, B.st.p, B.tiles.p, B.n_tiles, xi, par ^ 1);
    HIP_LAUNCH_OK();
    if (rbj) {
        ProfScope ps(prof ? ctx : nullptr, "rbj_apply", prof ? rbj_work(B) : 0.0);
        k_rbj_items<<<grid_of(B.n_rbj), TILE, 0, s>>>(B.tab.p, B.st.p, B.rbj.p, B.n_rbj);
        HIP_LAUNCH_OK();
    }
    k_cg_dir<<<grid_of(B.n_tiles), TILE, 0, s>>>(B.tab.p, B.st.p, B.tiles.p, B.n_tiles, par, 0,
                                                 prec == PCM_MIXED ? 1 : 0);
    HIP_LAUNCH_OK();
}

// GROUP_K iterations replayed from a captured graph (captured on first use and whenever the
// tables or the launch shape change)
static void launch_group(pcm_ctx *ctx, SolveBatch &B, int prec, int xi, int grid, bool rbj) {
    const int slot = prec == PCM_MIXED ? 1 : 0;
    GraphSig sig{B.tab.p, B.st.p, B.mv.p, B.tiles.p, B.rbj.p, B.n_mv, B.n_tiles, B.n_rbj, grid, rbj ? 1 : 0, prec};
    // xi is fixed per precision: FP64 solves x = V_XQ, mixed inner solves x = V_D
    if (!B.gexec[slot] || !(B.gsig[slot] == sig)) {
        if (B.gexec[slot]) HIP_OK(hipGraphExecDestroy(B.gexec[slot]));
        B.gexec[slot] = nullptr;
        if (!B.cap) HIP_OK(hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIP_OK(hipStreamBeginCapture(B.cap, hipStreamCaptureModeRelaxed));
        try {
            for (int g = 1; g <= GROUP_K; ++g) pcg_iteration(ctx, B, B.cap, prec, xi, g & 1, grid, rbj, false);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(B.cap, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        HIP_OK(hipStreamEndCapture(B.cap, &graph));
        hipError_t e = hipGraphInstantiate(&B.gexec[slot], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_OK(e);
        B.gsig[slot] = sig;
    }
    HIP_OK(hipGraphLaunch(B.gexec[slot], ctx->stream));
}

// PCG on A x = b for every molecule with act set (state already uploaded: act, tol, max_it);
// x = v[xi], b = v[bi].  Returns after every molecule has stopped.
static void pcg_batch(pcm_ctx *ctx, SolveBatch &B, int prec, int xi, int bi, bool zero_x, bool rbj) {
    hipStream_t s = ctx->stream;
    int max_it = 0;
    for (auto &h : B.h_st)
        if (h.act) max_it = std::max(max_it, h.max_it);
    const int grid = mv_grid(ctx, B, prec, 1, xi);
    if (!zero_x) matvec(ctx, B, s, PCM_FP64, 1, xi, V_Y, 0, 2, grid, ctx->prof);
    k_cg_init<<<grid_of(B.n_tiles), TILE, 0, s>>>(B.tab.p, B.st.p, B.tiles.p, B.n_tiles, xi, bi, zero_x ? 1 : 0);
    HIP_LAUNCH_OK();
    if (rbj) {
        k_rbj_items<<<grid_of(B.n_rbj), TILE, 0, s>>>(B.tab.p, B.st.p, B.rbj.p, B.n_rbj);
        HIP_LAUNCH_OK();
    }
    k_cg_dir<<<grid_of(B.n_tiles), TILE, 0, s>>>(B.tab.p, B.st.p, B.tiles.p, B.n_tiles, 0, 1,
                                                 prec == PCM_MIXED ? 1 : 0);
    HIP_LAUNCH_OK();
    if (ctx->prof) {
        // per-kernel profiling: one iteration at a time with the states read back after each,
        // so no launch runs after convergence and every record carries the work it did
        download_states(ctx, B);
        for (int g = 1; g <= max_it + 1; ++g) {
            bool any = false;
            for (const auto &h : B.h_st) any = any || takes_part(h, 0);
            if (!any) break;
            pcg_iteration(ctx, B, s, prec, xi, g & 1, grid, rbj, true);
            download_states(ctx, B);
        }
        return;
    }
    const int max_groups = max_it / GROUP_K + 2;
    // launch group j+1 before waiting for the active count of group j: the device never idles
    int launched = 0, slot = 0;
    auto group = [&](int sl) {
        launch_group(ctx, B, prec, xi, grid, rbj);
        k_count_active<<<1, TILE, 0, s>>>(B.st.p, B.n, B.cnt.p);
        HIP_LAUNCH_OK();
        HIP_OK(hipMemcpyAsync(B.h_cnt + sl, B.cnt.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_OK(hipEventRecord(B.ev[sl], s));
        ++launched;
    };
    // a molecule may already be done after the initial residual
    k_count_active<<<1, TILE, 0, s>>>(B.st.p, B.n, B.cnt.p);
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(B.h_cnt + 1, B.cnt.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipEventRecord(B.ev[1], s));
    HIP_OK(hipEventSynchronize(B.ev[1]));
    if (B.h_cnt[1] == 0) return;
    group(slot);
    while (true) {
        const int prev = slot;
        slot ^= 1;
        const bool more = launched < max_groups;
        if (more) group(slot);
        HIP_OK(hipEventSynchronize(B.ev[prev]));
        if (B.h_cnt[prev] == 0 || !more) break;
    }
}

// explicit residual v[V_RES] = b - A64 v[xi] and its squared norm into res2 (act molecules)
static void residual(pcm_ctx *ctx, SolveBatch &B, int xi, int bi) {
    const int grid = mv_grid(ctx, B, PCM_FP64, 1, xi);
    matvec(ctx, B, ctx->stream, PCM_FP64, 1, xi, V_RES, bi, 1, grid, ctx->prof);
    k_mol_reduce<<<B.n, TILE, 0, ctx->stream>>>(B.tab.p, B.st.p, 0);
    HIP_LAUNCH_OK();
}

static void vec_op(pcm_ctx *ctx, SolveBatch &B, int op, double a, int src, int dst,
                   const std::vector<const double *> *ext) {
    if (ext) HIP_OK(hipMemcpyAsync(B.ext.p, ext->data(), B.n * sizeof(double *), hipMemcpyHostToDevice, ctx->stream));
    k_vec_op<<<grid_of(B.n_tiles), TILE, 0, ctx->stream>>>(B.tab.p, B.st.p, B.tiles.p, B.n_tiles, op, a, src, dst,
                                                           B.ext.p);
    HIP_LAUNCH_OK();
}

static void dots3(pcm_ctx *ctx, SolveBatch &B, int a0, int b0, int a1, int b1, int a2, int b2) {
    k_dots3<<<grid_of(B.n_tiles), TILE, 0, ctx->stream>>>(B.tab.p, B.st.p, B.tiles.p, B.n_tiles, a0, b0, a1, b1, a2,
                                                          b2);
    HIP_LAUNCH_OK();
    k_mol_reduce<<<B.n, TILE, 0, ctx->stream>>>(B.tab.p, B.st.p, 1);
    HIP_LAUNCH_OK();
}

static void set_all(SolveBatch &B, int act, double tol, int max_it) {
    B.h_st.assign(B.n, CGState{});
    for (auto &h : B.h_st) {
        h.act = act;
        h.done = act ? 0 : 1;
        h.tol = tol;
        h.max_it = max_it;
    }
}

// Solve for every molecule of the batch.  v[i], q[i] are device vectors of molecule i.
pcm_status solve_batch_run(pcm_ctx *ctx, SolveBatch &B, const std::vector<const double *> &v,
                           const std::vector<double *> &q, const pcm_solve_opts &o, pcm_solve_info *info) {
    const int n = B.n;
    const double f = (ctx->prm.eps - 1.0) / (ctx->prm.eps + ctx->prm.k_factor);
    const bool blocks = o.precond == PCM_PRECOND_RBJ || o.precond == PCM_PRECOND_OCTREE;
    // work already queued on the stream (e.g. the esp that produced v) is not the solve's
    HIP_OK(hipStreamSynchronize(ctx->stream));
    auto t0 = std::chrono::steady_clock::now();
    for (pcm_mol *mol : B.mols) {
        solver_prepare(ctx, mol);
        if (blocks && mol->M > 0) rbj_setup(ctx, mol, o.precond, o.block, o.seed);
    }
    batch_tables(ctx, B, o.precond);
    std::vector<const double *> qc(q.begin(), q.end());
    set_all(B, 1, o.tol, o.max_iter);
    upload_states(ctx, B);
    vec_op(ctx, B, 0, 0.0, 0, V_V, &v);  // V = v
    if (o.warm_start)
        vec_op(ctx, B, 0, 0.0, 0, V_XQ, &qc);
    else
        vec_op(ctx, B, 4, 0.0, 0, V_XQ, nullptr);
    vec_op(ctx, B, 2, -f, V_V, V_B, nullptr);  // b = -f v
    HIP_OK(hipStreamSynchronize(ctx->stream));
    auto t1 = std::chrono::steady_clock::now();
    std::vector<int> iters(n, 0), refs(n, 0), conv(n, 0);
    std::vector<double> rn(n, 0.0);
    if (o.precision == PCM_MIXED) {
        // iterative refinement: r = b - A64 q; inner FP32-matvec PCG on A d = r; q += d
        const double eta = o.inner_rtol > 0 ? o.inner_rtol : 1e-4;
        std::vector<int> act(n, 1);
        while (true) {
            set_all(B, 0, o.tol, 0);
            for (int i = 0; i < n; ++i) B.h_st[i].act = act[i], B.h_st[i].done = 1;
            upload_states(ctx, B);
            residual(ctx, B, V_XQ, V_B);
            download_states(ctx, B);
            int n_act = 0;
            for (int i = 0; i < n; ++i) {
                if (!act[i]) continue;
                ++iters[i];
                rn[i] = std::sqrt(B.h_st[i].res2);
                if (rn[i] < o.tol) {
                    conv[i] = 1;
                    act[i] = 0;
                } else if (iters[i] >= o.max_iter || refs[i] > 200) {
                    act[i] = 0;
                }
                n_act += act[i];
            }
            if (!n_act) break;
            for (int i = 0; i < n; ++i) {
                CGState &h = B.h_st[i];
                h = CGState{};
                h.act = act[i];
                h.done = act[i] ? 0 : 1;
                h.tol = act[i] ? std::max(eta * rn[i], 0.5 * o.tol) : 0.0;
                h.max_it = act[i] ? std::min(o.max_iter - iters[i], INNER_MAX_IT) : 0;
            }
            upload_states(ctx, B);
            pcg_batch(ctx, B, PCM_MIXED, V_D, V_RES, true, blocks);
            vec_op(ctx, B, 3, 1.0, V_D, V_XQ, nullptr);  // q += d (act molecules)
            download_states(ctx, B);
            for (int i = 0; i < n; ++i)
                if (act[i]) {
                    iters[i] += B.h_st[i].it;
                    ++refs[i];
                }
        }
    } else {
        // The iteration runs on the recurrence residual; Eq. 20 is a test on b - A q itself,
        // so the recomputed residual decides, and a molecule whose recurrence converged while
        // its true residual did not restarts from the current q (a few times at most).
        std::vector<int> run(n, 1);
        bool first = true;
        for (int restart = 0; restart <= MAX_RESTARTS; ++restart) {
            pcg_batch(ctx, B, PCM_FP64, V_XQ, V_B, first ? !o.warm_start : false, blocks);
            download_states(ctx, B);
            std::vector<int> rec(n, 0);
            for (int i = 0; i < n; ++i)
                if (run[i]) {
                    iters[i] += B.h_st[i].it + (first && !o.warm_start ? 0 : 1);  // + the restart product
                    rec[i] = std::sqrt(B.h_st[i].rr) < o.tol;
                }
            for (int i = 0; i < n; ++i) B.h_st[i].act = run[i];
            upload_states(ctx, B);
            residual(ctx, B, V_XQ, V_B);
            download_states(ctx, B);
            int again = 0;
            for (int i = 0; i < n; ++i) {
                if (!run[i]) continue;
                rn[i] = std::sqrt(B.h_st[i].res2);
                conv[i] = rn[i] < o.tol;
                run[i] = rec[i] && !conv[i] && iters[i] < o.max_iter;
                again += run[i];
            }
            if (!again) break;
            first = false;
            for (int i = 0; i < n; ++i) {
                CGState &h = B.h_st[i];
                h = CGState{};
                h.act = run[i];
                h.done = run[i] ? 0 : 1;
                h.tol = o.tol;
                h.max_it = run[i] ? o.max_iter - iters[i] - 1 : 0;
            }
            upload_states(ctx, B);
        }
    }
    for (auto &h : B.h_st) h.act = 1;
    upload_states(ctx, B);
    vec_op(ctx, B, 1, 0.0, V_XQ, 0, &qc);  // q = XQ
    // Eq. 13 at q: v.q + 1/(2f) q.Aq with A q = b - res
    dots3(ctx, B, V_V, V_XQ, V_B, V_XQ, V_RES, V_XQ);
    download_states(ctx, B);
    auto t2 = std::chrono::steady_clock::now();
    bool all = true;
    for (int i = 0; i < n; ++i) {
        all = all && conv[i];
        if (!info) continue;
        pcm_solve_info &I = info[i];
        I.iters = iters[i];
        I.refinements = refs[i];
        I.resid = rn[i];
        const double *d = B.h_st[i].dots;
        I.energy = d[0] + 0.5 / f * (d[1] - d[2]);
        I.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        I.solve_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
    }
    return all ? PCM_OK : PCM_E_NOCONV;
}

// ----------------------------------------------------------------------------------------
// The batched solve as recorded launches for a captured graph: FP64 PCG from q = 0 with a fixed
// iteration budget (each molecule stops on the device when sqrt(r.r) < tol; its later
// iterations skip), the explicit residual, q copied out and the Eq. 13 energy.  All tables,
// the RBJ blocks and the matvec grid are set up now; the launches only read device memory.
// ----------------------------------------------------------------------------------------
struct GraphSolveBufs {
    DevBuf<const double *> bz, c, q;  // caller vectors per molecule
    DevBuf<CGState> init;             // the states every replay starts from
    ~GraphSolveBufs() {
        bz.release();
        c.release();
        q.release();
        init.release();
    }
};
GraphSolveBufs *graph_solve_bufs_new() { return new GraphSolveBufs(); }
void graph_solve_bufs_free(GraphSolveBufs *b) { delete b; }

__global__ void k_states_reset(CGState *__restrict__ st, const CGState *__restrict__ init, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) st[i] = init[i];
}

__global__ void k_energy_out(const CGState *__restrict__ st, int n, double half_inv_f, double *__restrict__ E) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) E[i] = st[i].dots[0] + half_inv_f * (st[i].dots[1] - st[i].dots[2]);
}

void solve_graph_launches(pcm_ctx *ctx, SolveBatch &B, const std::vector<const double *> &bz,
                          const std::vector<const double *> &c, const std::vector<double *> &q, double *E,
                          const pcm_solve_opts &o, int budget, GraphSolveBufs &gb, Launches &out) {
    const int n = B.n;
    const double f = (ctx->prm.eps - 1.0) / (ctx->prm.eps + ctx->prm.k_factor);
    const bool blocks = o.precond == PCM_PRECOND_RBJ || o.precond == PCM_PRECOND_OCTREE;
    for (pcm_mol *mol : B.mols) {
        solver_prepare(ctx, mol);
        if (blocks && mol->M > 0) rbj_setup(ctx, mol, o.precond, o.block, o.seed);
    }
    batch_tables(ctx, B, o.precond);
    auto ptrs = [&](DevBuf<const double *> &d, const std::vector<const double *> &h) {
        d.ensure(n);
        HIP_OK(hipMemcpyAsync(d.p, h.data(), n * sizeof(double *), hipMemcpyHostToDevice, ctx->stream));
    };
    ptrs(gb.bz, bz);
    ptrs(gb.c, c);
    ptrs(gb.q, std::vector<const double *>(q.begin(), q.end()));
    set_all(B, 1, o.tol, budget);
    upload_states(ctx, B);  // also the state the matvec grid is tuned with
    gb.init.ensure(n);
    HIP_OK(hipMemcpyAsync(gb.init.p, B.h_st.data(), n * sizeof(CGState), hipMemcpyHostToDevice, ctx->stream));
    const int grid = mv_grid(ctx, B, PCM_FP64, 1, V_XQ);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    SolveBatch *Bp = &B;
    const CGState *init = gb.init.p;
    const double *const *ebz = gb.bz.p, *const *ec = gb.c.p, *const *eq = gb.q.p;
    out.add("", 0.0, [=](hipStream_t st) {
        SolveBatch &b = *Bp;
        k_states_reset<<<div_up(n, 64), 64, 0, st>>>(b.st.p, init, n);
        HIP_LAUNCH_OK();
        const int gt = grid_of(b.n_tiles);
        k_vec_op<<<gt, TILE, 0, st>>>(b.tab.p, b.st.p, b.tiles.p, b.n_tiles, 0, 0.0, 0, V_V, ebz);  // v = Bz
        k_vec_op<<<gt, TILE, 0, st>>>(b.tab.p, b.st.p, b.tiles.p, b.n_tiles, 5, 0.0, 0, V_V, ec);   // v += c
        k_vec_op<<<gt, TILE, 0, st>>>(b.tab.p, b.st.p, b.tiles.p, b.n_tiles, 2, -f, V_V, V_B, ebz);  // b = -f v
        k_cg_init<<<gt, TILE, 0, st>>>(b.tab.p, b.st.p, b.tiles.p, b.n_tiles, V_XQ, V_B, 1);
        HIP_LAUNCH_OK();
        if (blocks) {
            k_rbj_items<<<grid_of(b.n_rbj), TILE, 0, st>>>(b.tab.p, b.st.p, b.rbj.p, b.n_rbj);
            HIP_LAUNCH_OK();
        }
        k_cg_dir<<<gt, TILE, 0, st>>>(b.tab.p, b.st.p, b.tiles.p, b.n_tiles, 0, 1, 0);
        HIP_LAUNCH_OK();
    });
    for (int g = 1; g <= budget; ++g)
        out.add("", 0.0, [=](hipStream_t st) { pcg_iteration(ctx, *Bp, st, PCM_FP64, V_XQ, g & 1, grid, blocks, false); });
    out.add("", 0.0, [=](hipStream_t st) {
        SolveBatch &b = *Bp;
        const int gt = grid_of(b.n_tiles);
        matvec(ctx, b, st, PCM_FP64, 1, V_XQ, V_RES, V_B, 1, grid, false);  // r = b - A q, |r|^2 partials
        k_mol_reduce<<<b.n, TILE, 0, st>>>(b.tab.p, b.st.p, 0);
        k_vec_op<<<gt, TILE, 0, st>>>(b.tab.p, b.st.p, b.tiles.p, b.n_tiles, 1, 0.0, V_XQ, 0, eq);  // q out
        // Eq. 13 at q: v.q + 1/(2f) q.Aq with A q = b - r
        k_dots3<<<gt, TILE, 0, st>>>(b.tab.p, b.st.p, b.tiles.p, b.n_tiles, V_V, V_XQ, V_B, V_XQ, V_RES, V_XQ);
        k_mol_reduce<<<b.n, TILE, 0, st>>>(b.tab.p, b.st.p, 1);
        k_energy_out<<<div_up(b.n, 64), 64, 0, st>>>(b.st.p, b.n, 0.5 / f, E);
        HIP_LAUNCH_OK();
    });
}

// per molecule after a replay: iterations, explicit residual and the convergence flag
void solve_graph_info(pcm_ctx *ctx, SolveBatch &B, double tol, pcm_solve_info *info, int *converged) {
    download_states(ctx, B);
    const double f = (ctx->prm.eps - 1.0) / (ctx->prm.eps + ctx->prm.k_factor);
    for (int i = 0; i < B.n; ++i) {
        const CGState &h = B.h_st[i];
        const double r = std::sqrt(h.res2);
        if (converged) converged[i] = r < tol || B.h_tab[i].M == 0;
        if (!info) continue;
        info[i] = pcm_solve_info{};
        info[i].iters = h.it;
        info[i].resid = r;
        info[i].energy = h.dots[0] + 0.5 / f * (h.dots[1] - h.dots[2]);
    }
}

static SolveBatch &solo(pcm_mol *mol) {
    if (!mol->solo) mol->solo = solve_batch_new({mol});
    return *mol->solo;
}

pcm_status run_solve(pcm_ctx *ctx, pcm_mol *mol, const double *vin, const pcm_solve_opts &o, double *q,
                     pcm_solve_info *info) {
    return solve_batch_run(ctx, solo(mol), {vin}, {q}, o, info);
}

// ----------------------------------------------------------------------------------------
// One rank's share of the product, the per-GPU kernel of the sharded matvec: the tile pairs
// (I, J >= I) whose position in the item order is rank mod nranks, plus A_kk x_k on the rows
// of the diagonal tile pairs it owns.  The shares of ranks 0 .. nranks-1 add up to A x.
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_share_finish(const CGMol *__restrict__ tab, int rank, int nranks, int src,
                                                       double *__restrict__ y) {
    const CGMol &m = tab[0];
    const int t = blockIdx.x, k = t * TILE + threadIdx.x;
    if (k >= m.M) return;
    double acc = 0.0;
    for (int r = 0; r < m.nT; ++r) acc += m.part[(size_t)r * m.M + k];
    const long long diag_item = (long long)t * m.nT - (long long)t * (t - 1) / 2;  // position of (t, t)
    if (diag_item % nranks == rank) acc += m.Akk[k] * m.v[src][k];
    y[k] = acc;
}

void run_matvec_share(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks) {
    SolveBatch &B = solo(mol);
    solver_prepare(ctx, mol);
    if (B.n_tiles == 0) batch_tables(ctx, B, PCM_PRECOND_NONE);
    set_all(B, 1, 0.0, 0);
    upload_states(ctx, B);
    std::vector<const double *> e_x{x};
    vec_op(ctx, B, 0, 0.0, 0, V_T, &e_x);
    const int nT = B.h_tab[0].nT, M = mol->M;
    std::vector<MvItem> items;
    long long pairs = 0;
    int idx = 0;
    for (int I = 0; I < nT; ++I)
        for (int J = I; J < nT; ++J, ++idx)
            if (idx % nranks == rank) {
                items.push_back(MvItem{0, I, J});
                const long long rI = std::min(TILE, M - I * TILE), rJ = std::min(TILE, M - J * TILE);
                pairs += I == J ? rI * (rI - 1) / 2 : rI * rJ;
            }
    B.share.ensure(std::max<size_t>(items.size(), 1));
    if (!items.empty())
        HIP_OK(hipMemcpyAsync(B.share.p, items.data(), items.size() * sizeof(MvItem), hipMemcpyHostToDevice,
                              ctx->stream));
    HIP_OK(hipMemsetAsync(B.part.p, 0, sizeof(double) * (size_t)nT * M, ctx->stream));
    if (!items.empty()) {
        ProfScope ps(ctx, "matvec_share_f64", (double)pairs);
        k_mv_sym<double><<<(int)items.size(), MV_THREADS, 0, ctx->stream>>>(B.tab.p, B.st.p, B.share.p,
                                                                             (int)items.size(), 1, V_T);
        HIP_LAUNCH_OK();
    }
    k_share_finish<<<nT, TILE, 0, ctx->stream>>>(B.tab.p, rank, nranks, V_T, y);
    HIP_LAUNCH_OK();
}

// E = bz.q + c.q + q.Aq / (2f)  (Eq. 13)
double run_energy(pcm_ctx *ctx, pcm_mol *mol, const double *bz, const double *c, const double *q) {
    SolveBatch &B = solo(mol);
    solver_prepare(ctx, mol);
    if (B.n_tiles == 0) batch_tables(ctx, B, PCM_PRECOND_NONE);  // item tables do not depend on precond
    const double f = (ctx->prm.eps - 1.0) / (ctx->prm.eps + ctx->prm.k_factor);
    set_all(B, 1, 0.0, 0);
    upload_states(ctx, B);
    std::vector<const double *> e_q{q}, e_bz{bz}, e_c{c};
    vec_op(ctx, B, 0, 0.0, 0, V_T, &e_q);
    vec_op(ctx, B, 0, 0.0, 0, V_V, &e_bz);
    vec_op(ctx, B, 0, 0.0, 0, V_RES, &e_c);
    const int grid = mv_grid(ctx, B, PCM_FP64, 1, V_T);
    matvec(ctx, B, ctx->stream, PCM_FP64, 1, V_T, V_Y, 0, 2, grid, ctx->prof);
    dots3(ctx, B, V_V, V_T, V_RES, V_T, V_T, V_Y);
    download_states(ctx, B);
    const double *d = B.h_st[0].dots;
    return d[0] + d[1] + 0.5 / f * d[2];
}

// ----------------------------------------------------------------------------------------
// Allocation-free share of the product (pcm_matvec_share_noalloc).  The kernels are those of
// run_matvec_share; every intermediate -- packed points, tile boxes, the copy of x, the item
// list, the molecule table and the partial slots -- lives in one fixed device array per GPU.
// Host code never names the array: its address on each device is looked up once, when a
// context first uses that device, and only that address is handed to kernels.
// ----------------------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[SCRATCH_MAX_DEV] = {};

void noalloc_scratch_init(int dev) {
    if (dev < 0 || dev >= SCRATCH_MAX_DEV) return;  // such a device has no allocation-free path
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
}

static unsigned char *noalloc_scratch(int dev) {
    if (dev < 0 || dev >= SCRATCH_MAX_DEV) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// byte offsets of the intermediates inside the scratch array (each 256-byte aligned)
struct NaLayout {
    size_t tab, st, items, p64, p32, tbox, x, part, total;
};
static size_t na_up(size_t b) { return (b + 255) / 256 * 256; }
static NaLayout na_layout(int M, long long n_items) {
    const size_t Mp = sv_pad(M), nT = Mp / TILE;
    NaLayout L{};
    size_t o = 0;
    L.tab = o;
    o += na_up(sizeof(CGMol));
    L.st = o;
    o += na_up(sizeof(CGState));
    L.items = o;
    o += na_up(sizeof(MvItem) * (size_t)std::max<long long>(n_items, 1));
    L.p64 = o;
    o += na_up(sizeof(Pt<double>) * Mp);
    L.p32 = o;
    o += na_up(sizeof(Pt<float>) * Mp);
    L.tbox = o;
    o += na_up(sizeof(double) * 6 * nT);
    L.x = o;
    o += na_up(sizeof(double) * Mp);
    L.part = o;
    o += na_up(sizeof(double) * nT * (size_t)M);
    L.total = o;
    return L;
}

// the molecule table and state of a one-molecule call, written from kernel arguments
__global__ void k_na_setup(CGMol m, CGState s, CGMol *__restrict__ tab, CGState *__restrict__ st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        tab[0] = m;
        st[0] = s;
    }
}

// item t of the share = tile pair at position rank + t * nranks of the (I, J >= I) order, whose
// row I starts at position I nT - I (I - 1) / 2
__global__ void k_na_items(MvItem *__restrict__ out, int nT, int rank, int nranks, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const long long p = rank + (long long)t * nranks;
    int lo = 0, hi = nT - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((long long)mid * nT - (long long)mid * (mid - 1) / 2 <= p) lo = mid;
        else hi = mid - 1;
    }
    const long long s = (long long)lo * nT - (long long)lo * (lo - 1) / 2;
    out[t] = MvItem{0, lo, lo + (int)(p - s)};
}

// x copied into an Mp-long vector with a zero tail; partial slots cleared (a share writes only
// the slots of its own tile pairs)
__global__ void k_na_prep(const double *__restrict__ x, double *__restrict__ xv, int M, int Mp,
                          double *__restrict__ part, long long n_part) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Mp) xv[i] = i < M ? x[i] : 0.0;
    for (long long k = i; k < n_part; k += (long long)gridDim.x * blockDim.x) part[k] = 0.0;
}

long long noalloc_scratch_bytes() { return (long long)SCRATCH_BYTES; }

void run_matvec_share_noalloc(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks) {
    const int M = mol->M, Mp = sv_pad(M), nT = Mp / TILE;
    const long long n_pos = (long long)nT * (nT + 1) / 2;
    const long long n_items = rank < n_pos ? (n_pos - rank + nranks - 1) / nranks : 0;
    const NaLayout L = na_layout(M, n_items);
    if (L.total > SCRATCH_BYTES)
        throw PcmError{PCM_E_ARG, "M = " + std::to_string(M) + " needs " + std::to_string(L.total) +
                                      " bytes of scratch; the allocation-free product holds " +
                                      std::to_string(SCRATCH_BYTES) + " (about M <= 45,000)"};
    unsigned char *base = noalloc_scratch(ctx->device);
    if (!base) throw PcmError{PCM_E_STATE, "no scratch address for this device (context not initialised)"};
    if (M == 0) return;
    CGMol *tab = reinterpret_cast<CGMol *>(base + L.tab);
    CGState *st = reinterpret_cast<CGState *>(base + L.st);
    MvItem *items = reinterpret_cast<MvItem *>(base + L.items);
    Pt<double> *p64 = reinterpret_cast<Pt<double> *>(base + L.p64);
    Pt<float> *p32 = reinterpret_cast<Pt<float> *>(base + L.p32);
    double *tbox = reinterpret_cast<double *>(base + L.tbox);
    double *xv = reinterpret_cast<double *>(base + L.x);
    double *part = reinterpret_cast<double *>(base + L.part);
    CGMol m{};
    m.v[V_T] = xv;
    m.pt64 = p64;
    m.pt32 = p32;
    m.Akk = mol->Akk.p;
    m.part = part;
    m.tbox = tbox;
    m.boys64 = ctx->boys64.p;
    m.boys32 = ctx->boys32.p;
    double r32;
    mv_cutoffs(mol, m.rc2_64, r32);
    m.rc2_32 = (float)r32;
    m.M = M;
    m.Mp = Mp;
    m.nT = nT;
    m.ndp = nT;
    m.n_rz = nT;
    m.precond = PCM_PRECOND_NONE;
    CGState s{};
    s.act = 1;
    s.done = 1;
    hipStream_t stm = ctx->stream;
    k_na_setup<<<1, 64, 0, stm>>>(m, s, tab, st);
    HIP_LAUNCH_OK();
    k_pack_pts<<<grid_for(Mp, 256), 256, 0, stm>>>(mol->px.p, mol->py.p, mol->pz.p, mol->zeta.p, M, Mp, p64, p32);
    HIP_LAUNCH_OK();
    k_tile_box<<<nT, TILE, 0, stm>>>(p64, M, tbox);
    HIP_LAUNCH_OK();
    const long long n_part = (long long)nT * M;
    k_na_prep<<<std::max(grid_for(Mp, 256), 1024), 256, 0, stm>>>(x, xv, M, Mp, part, n_part);
    HIP_LAUNCH_OK();
    if (n_items > 0) {
        k_na_items<<<grid_for(n_items, 256), 256, 0, stm>>>(items, nT, rank, nranks, (int)n_items);
        HIP_LAUNCH_OK();
        k_mv_sym<double><<<(int)n_items, MV_THREADS, 0, stm>>>(tab, st, items, (int)n_items, 1, V_T);
        HIP_LAUNCH_OK();
    }
    k_share_finish<<<nT, TILE, 0, stm>>>(tab, rank, nranks, V_T, y);
    HIP_LAUNCH_OK();
}
