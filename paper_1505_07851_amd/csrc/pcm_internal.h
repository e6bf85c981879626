// Internal declarations of the gfx950 C-PCM library: handle layouts, launch helpers
// and the device math shared by the integral, solver and gradient kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/pcm.h"
#include "hermite_gen.h"

// ----------------------------------------------------------------------------------------
// error plumbing
// ----------------------------------------------------------------------------------------
struct PcmError {
    pcm_status st;
    std::string msg;
};

#define HIP_OK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw PcmError{PCM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)};      \
    } while (0)

// failure with a message kept in the context; calls wrapped in guarded() turn exceptions into
// status codes (nothing throws across the C ABI)
inline pcm_status fail(pcm_ctx *ctx, pcm_status st, const std::string &msg);
template <typename F> pcm_status guarded(pcm_ctx *ctx, F &&f);

#define HIP_LAUNCH_OK()                                                                        \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess)                                                                  \
            throw PcmError{PCM_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)}; \
    } while (0)

// ----------------------------------------------------------------------------------------
// classes of shell pairs (Sec. 4a: ss, sp, sd, pp, pd, dd)
// ----------------------------------------------------------------------------------------
constexpr int NCLS = 6;
constexpr int CLS_LA[NCLS] = {0, 0, 0, 1, 1, 2};
constexpr int CLS_LB[NCLS] = {0, 1, 2, 1, 2, 2};
__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
__host__ __device__ constexpr int ntuv(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
// position of (t,u,v) in the order: N = t+u+v ascending, t descending, u descending
__host__ __device__ constexpr int tuv_idx(int t, int u, int v) {
    int N = t + u + v;
    return N * (N + 1) * (N + 2) / 6 + (N - t) * (N - t + 1) / 2 + (N - t - u);
}
// Cartesian component c of shell l in lexicographic order (x, y, z; xx, xy, xz, yy, yz, zz)
__host__ __device__ inline void cart_comp(int l, int c, int &ax, int &ay, int &az) {
    int n = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (n == c) { ax = x; ay = y; az = l - x - y; return; }
            ++n;
        }
    ax = ay = az = 0;
}

// ----------------------------------------------------------------------------------------
// Boys function tables.  F_m(T_i) at T_i = i/8; Taylor expansion around the nearest node:
// F_m(T) = sum_k F_{m+k}(T_i) (T_i - T)^k / k!.  FP64: order 8 on [0, 40); FP32: order 4 on
// [0, 30).  Above the range the asymptotic form is used, whose neglected tail is bounded in
// aux_Rn (below 2e-12 relative at T = 40 for the orders used here).
// ----------------------------------------------------------------------------------------
template <typename T> struct BoysCfg;
template <> struct BoysCfg<double> {
    static constexpr int ORD = 8, MT = 14, NROW = 321;
    static constexpr double TMAX = 40.0;
};
template <> struct BoysCfg<float> {
    // rows up to T = 40: the mixed kernels interpolate in FP32 over the FP64 kernels' near range
    // [0, 40); the all-FP32 kernels switch to the asymptotic form at 30
    static constexpr int ORD = 4, MT = 10, NROW = 321;
    static constexpr float TMAX = 30.0f;
};
constexpr int LMAX_TOT = 5;  // highest total L handled (d-d gradient)

// ----------------------------------------------------------------------------------------
// Pair records.  A "header" holds the Gaussian-product data of one primitive pair:
//   P (double), p, TMAX/p (far-field test), (pi/p)^{3/2} (far prefactor), 2 pi/p (near).
// The density-contracted Hermite coefficients D_tuv follow for the esp/gradient lists.
// ----------------------------------------------------------------------------------------
template <typename T> struct PairHdr {
    double Px, Py, Pz;
    T p, limp, pf, pref;
};
__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
template <typename T> __host__ __device__ constexpr size_t rec_stride(int L) {
    return align16(sizeof(PairHdr<T>) + sizeof(T) * ntuv(L));
}

// ----------------------------------------------------------------------------------------
// Auxiliary values R^(n)_000 (n = 0..L) of one (pair, point) evaluation, prefactors included.
//   near: (2 pi/p) sqrt(u) (-2 a)^n F_n(a r^2),  u = z^2/(z^2+p), a = p u;
//   far (a r^2 >= TMAX): the smeared charge acts as a point charge and the attenuation
//   drops out: (pi/p)^{3/2} (-1)^n (2n-1)!! / r^{2n+1}.  The terms left out are bounded by the
//   upper incomplete gamma tail, e^{-T} T^{n-1/2} / Gamma(n+1/2) relative to F_n(T): below
//   2e-12 at T = 40 for n <= 5 (FP64 and mixed kernels), below 1e-8 at T = 30 (FP32 kernels).
// The far test a r^2 >= TMAX is r^2 >= TMAX/p + TMAX/z^2.
//
// Precisions: T is the type of the pair records, the far field and the accumulation, B the type
// of the Boys-table interpolation of the near field.
//   T = B = double: FP64 throughout.
//   T = double, B = float (mixed): the near-field Taylor interpolation of F_n(T) runs in FP32 on
//     the FP32 table (order 4); its argument, the prefactors and the scaling to R^(n) stay FP64,
//     and the large-T branch is FP64.
//   T = B = float: FP32 throughout (used only for pairs whose screening bound is small).
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return rsqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }

// 1/sqrt(x) for finite x > 0: hardware estimate refined by one cubic correction step,
// y = y0 (1 - e)^(-1/2) ~ y0 (1 + e/2 + 3e^2/8) with e = 1 - x y0^2.
__device__ __forceinline__ double rsq_fast(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float rsq_fast(float x) { return __builtin_amdgcn_rsqf(x); }

// Surface point as the integral kernels read it (wave-uniform in the pair-per-lane kernels):
// position in FP64 (differences P - C are taken in FP64 in both precisions), the exponent
// zeta, its square and the far-field limit TMAX / zeta^2 in the kernel's precision.
template <typename T> struct PtInt {
    double x, y, z;
    T zeta2, zeta, lim;
};
constexpr int PT_PAD = 64;  // point arrays are padded to a multiple of this with far dummies

// Columns of the LDS copy of the Boys table a kernel needs: F_0 .. F_{L+ORD} for R^(n),
// n <= L.  Kernels stage only these columns, so low-L kernels keep more workgroups resident.
template <typename T, int L> __host__ __device__ constexpr int boys_cols() { return L + BoysCfg<T>::ORD + 1; }

// near field (a r^2 < TMAX) of aux_Rn: the Boys-table interpolation
template <int L, typename T, typename B = T>
__device__ __forceinline__ void aux_Rn_near(T r2, T p, T pref, T zeta2, T zeta, const B *__restrict__ tab,
                                            T (&Rn)[L + 1]) {
    using C = BoysCfg<B>;
    static_assert(boys_cols<B, L>() <= C::MT, "Boys table has too few columns for this L");
    // sqrt(u) = zeta / sqrt(zeta^2 + p), u = sqrt(u)^2, a = p u
    T su = zeta * rsq_fast(zeta2 + p);
    T u = su * su;
    T a = p * u;
    T tb = a * r2;
    int i = (int)(tb * T(8) + T(0.5));
    i = i < C::NROW - 1 ? i : C::NROW - 1;
    const B d = (B)(T(i) * T(0.125) - tb);
    // F_n(T) = sum_k F_{n+k}(T_i) d^k / k!, nested: F_n + d (F_{n+1} + d/2 (F_{n+2} + ...)),
    // in the table's precision
    B dk[C::ORD + 1];
#pragma unroll
    for (int k = 1; k <= C::ORD; ++k) dk[k] = d * (B(1) / B(k));
    const B *row = tab + i * boys_cols<B, L>();
    T fac = pref * su;
    T m2a = T(-2) * a;
#pragma unroll
    for (int n = 0; n <= L; ++n) {
        B F = row[n + C::ORD];
#pragma unroll
        for (int k = C::ORD; k >= 1; --k) F = fma(F, dk[k], row[n + k - 1]);
        Rn[n] = fac * (T)F;
        fac *= m2a;
    }
}

template <int L, typename T, typename B = T>
__device__ __forceinline__ void aux_Rn(T r2, T p, T limp, T pf, T pref, T zeta2, T zeta, T limk,
                                       const B *__restrict__ tab, T (&Rn)[L + 1]) {
    if (r2 >= limp + limk) {
        T ri = rsq_fast(r2);
        T ri2 = ri * ri;
        Rn[0] = pf * ri;
#pragma unroll
        for (int n = 1; n <= L; ++n) Rn[n] = T(-(2 * n - 1)) * ri2 * Rn[n - 1];
    } else {
        aux_Rn_near<L, T, B>(r2, p, pref, zeta2, zeta, tab, Rn);
    }
}

// R_tuv (t+u+v <= L) of one pair against one point; (X, Y, Z) = P - C.
template <int L, typename T, typename B = T>
__device__ __forceinline__ void eval_R(double X, double Y, double Z, const PairHdr<T> &h, T zeta2, T zeta, T limk,
                                       const B *__restrict__ tab, T (&R)[ntuv(L)]) {
    T x = T(X), y = T(Y), z = T(Z);
    T r2 = x * x + y * y + z * z;
    T Rn[L + 1];
    aux_Rn<L, T, B>(r2, h.p, h.limp, h.pf, h.pref, zeta2, zeta, limk, tab, Rn);
    MdR<L>::run(x, y, z, Rn, R);
}

// name of a kernel precision (records/accumulation T, Boys interpolation B) in profiles and keys
template <typename T, typename B> constexpr const char *prec_tag() {
    return sizeof(T) == 4 ? "f32" : (sizeof(B) == 4 ? "mix" : "f64");
}

// pairs per batch of wave-uniform record loads in the point-per-lane kernels
template <int L> __host__ __device__ constexpr int pair_batch() { return L == 0 ? 4 : (L <= 2 ? 2 : 1); }
// Pair batch of the point-side kernels that request the next batch's records during the current
// evaluation (classes with L <= 2): both batches of records fit in the scalar registers (at L = 1
// with a few scalars of the item set aside in vector lanes outside the pair loop)
template <int L> __host__ __device__ constexpr int pair_batch_pf() { return L <= 1 ? 2 : 1; }

// Empty statements that need a wave-uniform value in scalar registers at this point: a scalar load
// of it must have completed here (the compiler places its wait just before)
template <typename T> __device__ __forceinline__ void pin_sgpr(const T &v) { asm volatile("" ::"s"(v)); }
template <typename T> __device__ __forceinline__ void pin_sgpr(const PairHdr<T> &h) {
    pin_sgpr(h.Px);
    pin_sgpr(h.Py);
    pin_sgpr(h.Pz);
    pin_sgpr(h.p);
    pin_sgpr(h.limp);
    pin_sgpr(h.pf);
    pin_sgpr(h.pref);
}
constexpr int REC_PAD = 4;  // pair record lists are padded to a multiple of this with zero records
constexpr int PT_BATCH = 4; // points per batch in the pair-per-lane kernels

// DPP moves within a row of 16 lanes (VALU only, no LDS round trip)
constexpr int DPP_ROW_ROR8 = 0x128;     // lane i <- lane (i + 8) mod 16: partner differs in bit 3
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane i <- lane 7 - i within 8: partner differs in bit 2
constexpr int DPP_QUAD_XOR2 = 0x4E;     // quad_perm [2, 3, 0, 1]
constexpr int DPP_QUAD_XOR1 = 0xB1;     // quad_perm [1, 0, 3, 2]

// Every lane of every row and bank is written and every source lane exists for these
// patterns, so no "old" operand is needed.
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Read-only view through the constant address space: wave-uniform loads from it become
// scalar loads.  Only for data that no thread of the running kernel writes.  (The host pass
// of the compiler only type-checks these declarations.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using cptr = const __attribute__((address_space(4))) T *;
#else
template <typename T> using cptr = const T *;
#endif
template <typename T> __device__ __forceinline__ cptr<T> as_const(const T *p) { return (cptr<T>)(p); }

// descriptor of work item `it` in a table sorted by first item `base` (batched launches; `it`
// may differ between lanes, as in the per-pair contraction kernels)
template <typename D> __device__ __forceinline__ int find_desc(const D *__restrict__ ds, int nd, long long it) {
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (ds[mid].base <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Stage the Boys columns an order-L evaluation reads into LDS (row stride boys_cols<T, L>);
// tab_g holds BoysCfg<T>::NROW rows of MT values.
template <typename T, int L>
__device__ __forceinline__ void load_boys(T *lds, const T *__restrict__ tab_g) {
    constexpr int NC = boys_cols<T, L>(), n = BoysCfg<T>::NROW * NC;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int row = i / NC, col = i - row * NC;
        lds[i] = tab_g[row * BoysCfg<T>::MT + col];
    }
    __syncthreads();
}
template <typename T, int L> constexpr int boys_lds_size() { return BoysCfg<T>::NROW * boys_cols<T, L>(); }

// ----------------------------------------------------------------------------------------
// 1-D Hermite expansion coefficients of a Cartesian Gaussian product (without the
// exponential prefactor): E[i][j][t] for i <= IM, j <= JM,
//   E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1}, and likewise for j.
// ----------------------------------------------------------------------------------------
template <int IM, int JM>
struct Herm1D {
    double e[IM + 1][JM + 1][IM + JM + 1];
    __device__ void build(double PA, double PB, double inv2p) {
        for (int i = 0; i <= IM; ++i)
            for (int j = 0; j <= JM; ++j)
                for (int t = 0; t <= IM + JM; ++t) e[i][j][t] = 0.0;
        e[0][0][0] = 1.0;
        for (int i = 0; i <= IM; ++i) {
            if (i > 0)
                for (int t = 0; t <= i; ++t) {
                    double v = PA * e[i - 1][0][t];
                    if (t > 0) v += inv2p * e[i - 1][0][t - 1];
                    if (t + 1 <= i - 1) v += (t + 1) * e[i - 1][0][t + 1];
                    e[i][0][t] = v;
                }
            for (int j = 1; j <= JM; ++j)
                for (int t = 0; t <= i + j; ++t) {
                    double v = PB * e[i][j - 1][t];
                    if (t > 0) v += inv2p * e[i][j - 1][t - 1];
                    if (t + 1 <= i + j - 1) v += (t + 1) * e[i][j - 1][t + 1];
                    e[i][j][t] = v;
                }
        }
    }
};

// The same coefficients built in LDS by one lane (runtime indices), for kernels that give a
// whole wave to one primitive pair: e[(i * (JM + 1) + j) * (IM + JM + 1) + t].
template <int IM, int JM> constexpr int herm1d_size() { return (IM + 1) * (JM + 1) * (IM + JM + 1); }
template <int IM, int JM>
__device__ void herm1d_build_lds(double *e, double PA, double PB, double inv2p) {
    constexpr int TS = IM + JM + 1;
    auto E = [&](int i, int j, int t) -> double & { return e[(i * (JM + 1) + j) * TS + t]; };
    for (int x = 0; x < herm1d_size<IM, JM>(); ++x) e[x] = 0.0;
    E(0, 0, 0) = 1.0;
    for (int i = 0; i <= IM; ++i) {
        if (i > 0)
            for (int t = 0; t <= i; ++t) {
                double v = PA * E(i - 1, 0, t);
                if (t > 0) v += inv2p * E(i - 1, 0, t - 1);
                if (t + 1 <= i - 1) v += (t + 1) * E(i - 1, 0, t + 1);
                E(i, 0, t) = v;
            }
        for (int j = 1; j <= JM; ++j)
            for (int t = 0; t <= i + j; ++t) {
                double v = PB * E(i, j - 1, t);
                if (t > 0) v += inv2p * E(i, j - 1, t - 1);
                if (t + 1 <= i + j - 1) v += (t + 1) * E(i, j - 1, t + 1);
                E(i, j, t) = v;
            }
    }
}

// ----------------------------------------------------------------------------------------
// host-side handles
// ----------------------------------------------------------------------------------------
template <typename T> struct DevBuf {
    T *p = nullptr;
    size_t n = 0;  // capacity in elements
    void ensure(size_t want) {
        if (want <= n && p) return;
        if (p) HIP_OK(hipFree(p));
        p = nullptr;
        n = 0;
        if (want == 0) return;
        if (hipMalloc(&p, want * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw PcmError{PCM_E_ALLOC, "device allocation of " + std::to_string(want * sizeof(T)) + " bytes failed"};
        }
        n = want;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// per-kernel timing with HIP events on the context stream (enabled by pcm_profile_enable)
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
    double work;
};
struct ProfAgg {
    std::string name;
    double ms;
    long long launches;
    double work;
};

struct pcm_ctx {
    pcm_params prm{};
    bool prof = false;
    std::vector<ProfRec> prof_recs;
    std::vector<ProfAgg> prof_agg;
    hipStream_t stream = nullptr;
    int device = -1;
    bool dev_ready = false;
    std::string err;
    DevBuf<double> boys64;
    DevBuf<float> boys32;
    DevBuf<double> scal;  // small scalar workspace (reductions, solver scalars)
    DevBuf<int> iscal;
    DevBuf<long long> lscal;
    std::map<std::string, int> tuned;  // autotuner choices by kernel / shape key
    DevBuf<unsigned char> desc;        // descriptor tables of the current integral launch
};

// Time launch(c) for every candidate c (one warm-up, then the best of `reps` timed runs on
// the context stream) and return the fastest; the choice is cached under `key`.
int autotune_pick(pcm_ctx *ctx, const std::string &key, const std::vector<int> &cands,
                  const std::function<void(int)> &launch, int reps = 2);

// one screened primitive-pair list (all classes, concatenated by class)
struct PairList {
    long long cls_off[NCLS + 1] = {0};  // prim-pair offsets per class
    long long sp_count[NCLS] = {0};     // shell pairs with at least one surviving primitive pair
    long long sp_union[NCLS] = {0};     // the same before a precision split (both parts together)
    long long n = 0;
    DevBuf<int> spo;        // [n_sp_cand + 1] exclusive prefix of surviving counts per candidate
    DevBuf<int> cnt;        // [n_sp_cand] surviving count per candidate shell pair
    DevBuf<unsigned long long> mask;  // [n_sp_cand] surviving (i,j) bit mask
    DevBuf<int> ent_sp, ent_ij;       // [n] candidate shell pair index, i*8+j
    DevBuf<unsigned char> rec;        // pair records (type and stride depend on use)
    size_t rec_off[NCLS + 1] = {0};   // byte offsets of each class in rec
    // [n] per class, the class-local record index each lane of a pair-per-lane kernel takes: the
    // records grouped by exponent, then along a Morton curve of the product centre, so that a
    // wave's pairs are alike in p and close together and the near-field branch is taken by fewer
    // waves.  The kernels write their per-pair sums in this order (slot = lane), and the
    // contraction kernels that read them walk the same slots and write per list entry.  Results
    // do not depend on this order.
    DevBuf<int> vperm;
};

// the pair order of class cl for the pair-per-lane kernels (null when the list has none)
inline const int *pair_order(const PairList &pl, int cl) {
    return pl.vperm.p && pl.cls_off[cl + 1] > pl.cls_off[cl] ? pl.vperm.p + pl.cls_off[cl] : nullptr;
}

struct SolveBatch;
struct RbjPending;
struct pcm_graph;

struct pcm_mol {
    int N = 0, nsph = 0, M = 0, Mraw = 0;
    double zeta0 = 4.9;
    int ns = 0, nbf = 0, nprim = 0;
    // host copies
    std::vector<double> h_xyz, h_Z, h_rad, h_dirs, h_w;
    std::vector<int> h_sl, h_snp, h_soff, h_satom, h_bf, h_cnoff;
    std::vector<double> h_pexp, h_pcoef;
    std::vector<int> h_keep;  // kept raw indices (atom * nsph + j)
    // device: atoms and sphere rule
    DevBuf<double> xyz, Z, rad, dirs, w;
    // device: basis
    DevBuf<int> sl, snp, soff, satom, bfo, cnoff;
    DevBuf<double> pexp, pcoef, cn;
    // device: surface (SoA, FP64) and packed point records
    DevBuf<int> keep;  // [M]
    DevBuf<double> px, py, pz, zeta, S, Akk;
    int Mpad = 0;                     // M rounded up to PT_PAD
    DevBuf<unsigned char> pti64;      // [Mpad] PtInt<double> (far dummies past M)
    DevBuf<unsigned char> pti32;      // [Mpad] PtInt<float>
    DevBuf<double> qpad;              // [Mpad] charges copied for the point loops (zeros past M)
    DevBuf<double> r_surf_buf;        // [3M] explicit surface positions of pcm_update_geometry
    // candidate shell pairs (classes concatenated)
    long long sp_cls_off[NCLS + 1] = {0};
    std::vector<int> h_spa, h_spb;
    DevBuf<int> spa, spb;
    // per-atom lists of candidate shell pairs (CSR) for the gradient reduction
    DevBuf<int> atom_sp_off_a, atom_sp_a, atom_sp_off_b, atom_sp_b;
    // screened lists; with PCM_DYNAMIC precision fock / esp hold the pairs whose bound reaches
    // dp_thresh (FP64 records) and fock_w / esp_w the others (FP32 records), both in list order
    PairList fock, esp, fock_w, esp_w;
    // lists of the one-pass Fock + gradient pair side (header-only records): fg holds the Eq. 18
    // survivors for the current P (V' up to L + 1 feeds the gradient and, for its Eq. 15 members,
    // the Fock matrix), fo the Eq. 15 survivors outside Eq. 18 (V up to L, Fock only)
    PairList fg, fg_w;                  // fg_w: the FP32 part of a PCM_DYNAMIC split (else empty)
    PairList fo, fo_w;                  // fo_w: likewise
    DevBuf<unsigned long long> m18, m15;  // Eq. 18 and Eq. 15 survivor bits per candidate shell pair
    DevBuf<int> c18;
    DevBuf<unsigned long long> mtmp;    // screening scratch of the precision splits [3 x candidates]
    DevBuf<int> ctmp;
    DevBuf<int> pperm;                  // [M] point taken by each lane of the point-per-lane kernels
    DevBuf<unsigned> okey;              // pair-order sort scratch: keys in and out [2 x entries]
    DevBuf<int> oval;                   // class-local indexes to sort [entries]
    DevBuf<unsigned char> osort;        // radix sort temporary storage
    bool esp_valid = false;
    // workspaces
    DevBuf<double> part;   // partial sums (esp / gradient)
    DevBuf<double> vbuf;   // V_tuv partials (fock / grad)
    DevBuf<double> fprim;  // per prim pair Fock blocks
    DevBuf<double> gpair;  // per prim pair gradient contributions
    DevBuf<double> gsp;    // per candidate shell pair gradient sums
    DevBuf<int> scan_tmp;
    // solver
    DevBuf<double> sv;     // solver vectors, packed points
    SolveBatch *solo = nullptr;  // solver tables of this molecule alone
    DevBuf<double> rbj_inv;
    DevBuf<int> rbj_perm, rbj_off;
    DevBuf<long long> rbj_ioff;
    std::vector<int> h_rbj_perm, h_rbj_off;
    int rbj_kind = 0, rbj_l = -1, rbj_lmax = 0;
    RbjPending *rbj_pending = nullptr;  // partition started on a host thread after a geometry update
    unsigned long long rbj_seed = 0;
    bool rbj_valid = false;
    pcm_ctx *owner_ctx = nullptr;
    pcm_graph *graph = nullptr;  // a captured graph that holds this molecule's buffers (calls refused)
};

struct pcm_batch {
    std::vector<pcm_mol *> mols;
    SolveBatch *solve = nullptr;
    pcm_graph *graph = nullptr;
};

// which list of a molecule a kernel sequence reads
using ListSel = PairList pcm_mol::*;

inline pcm_status fail(pcm_ctx *ctx, pcm_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

template <typename F> pcm_status guarded(pcm_ctx *ctx, F &&f) {
    try {
        pcm_status st = f();
        if (st == PCM_OK && ctx) ctx->err.clear();
        return st;
    } catch (const PcmError &e) {
        return fail(ctx, e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(ctx, PCM_E_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(ctx, PCM_E_HIP, "unexpected failure");
    }
}

// API helpers shared by the C-ABI units (api.hip, graph.hip)
pcm_status check_solve_opts(pcm_ctx *ctx, const pcm_solve_opts *opts, pcm_solve_opts &o);
pcm_status density_list(pcm_ctx *ctx, pcm_mol *mol, const double *P);

// records one launch (or a short sequence) between construction and destruction
struct ProfScope {
    pcm_ctx *c;
    ProfRec r{};
    bool on;
    ProfScope(pcm_ctx *ctx, const std::string &name, double work) : c(ctx), on(ctx && ctx->prof) {
        if (!on) return;
        r.name = name;
        r.work = work;
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess ||
            hipEventRecord(r.a, c->stream) != hipSuccess)
            on = false;
    }
    ~ProfScope() {
        if (on && hipEventRecord(r.b, c->stream) == hipSuccess) c->prof_recs.push_back(r);
    }
};

// A recorded sequence of kernel launches: the host work of a pass (screening, chunk choice,
// descriptor uploads) is done when the sequence is built, so running it only launches kernels
// (immediately on the context's stream, or under capture into a hipGraph).
struct Launch {
    std::string name;  // profiling name ("" = not profiled)
    double work;
    std::function<void(hipStream_t)> fn;
};
struct Launches {
    std::vector<Launch> v;
    void add(const std::string &name, double work, std::function<void(hipStream_t)> fn) {
        v.push_back(Launch{name, work, std::move(fn)});
    }
    // prof: wrap each named launch in HIP events on the context's stream (immediate runs only)
    void run(pcm_ctx *ctx, hipStream_t s, bool prof) const {
        for (const Launch &l : v) {
            if (prof && !l.name.empty()) {
                ProfScope ps(ctx, l.name, l.work);
                l.fn(s);
            } else {
                l.fn(s);
            }
        }
    }
};

// ----------------------------------------------------------------------------------------
// internal entry points implemented in the .hip translation units
// ----------------------------------------------------------------------------------------
void ctx_ensure_device(pcm_ctx *ctx);
void scan_exclusive(pcm_ctx *ctx, pcm_mol *mol, const int *in, int *out, long long n, long long *total);
void surface_build(pcm_ctx *ctx, pcm_mol *mol, bool prune);
void basis_normalise(pcm_ctx *ctx, pcm_mol *mol);
void pairs_build(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P, int kind /*0 fock, 1 esp*/);
void pairs_prepare_geometry(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, int prec);
void pairs_prepare_density(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P, int prec);
// keep in `pl` the survivors whose Eq. 15 bound (times max |P| when P is given) reaches thresh,
// move the others to `weak`; both keep the list order
void pairs_split(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, PairList &weak, const double *P, double thresh);
void run_bz(pcm_ctx *ctx, pcm_mol *mol, double *bz);
// Recorded launches (no host work when run) of the passes a captured graph replays
void bz_launches(pcm_ctx *ctx, pcm_mol *mol, double *bz, Launches &out);
void density_record_launches(pcm_ctx *ctx, pcm_mol *mol, PairList &pl, const double *P, int prec, Launches &out);
void esp_batch_launches(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<double *> &c, int prec,
                        std::vector<std::unique_ptr<DevBuf<unsigned char>>> &bufs, Launches &out);
void fock_batch_launches(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &q,
                         const std::vector<double *> &F, int prec,
                         std::vector<std::unique_ptr<DevBuf<unsigned char>>> &bufs, Launches &out);
void run_esp(pcm_ctx *ctx, pcm_mol *mol, double *c, int prec);
void run_fock(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F, int prec);
void run_esp_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<double *> &c, int prec);
void run_fock_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &q,
                    const std::vector<double *> &F, int prec);
pcm_status run_solve(pcm_ctx *ctx, pcm_mol *mol, const double *v, const pcm_solve_opts &o, double *q,
                     pcm_solve_info *info);
double run_energy(pcm_ctx *ctx, pcm_mol *mol, const double *bz, const double *c, const double *q);
void run_matvec_share(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks);
// the same share with every intermediate in the fixed per-device scratch array (no allocation)
void run_matvec_share_noalloc(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks);
// look up (once per device, with that device current) the address of the scratch array
void noalloc_scratch_init(int dev);
long long noalloc_scratch_bytes();
void run_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, double *g_nuc, double *g_surf,
              int prec);
// c (Eqs. 5-6) and dc_k = d c_k / d r_k (M x 3) in one pass over the Eq. 18 list(s): the point
// side of the Eq. 22 gradient with the potential accumulated beside it
void run_esp_deriv(pcm_ctx *ctx, pcm_mol *mol, double *c, double *dc, int prec);
// F += L^T q (Eq. 10) and the Eq. 14 gradient with the c term's point side from dc: one pair-side
// pass over the Eq. 18 list fg for both, and the Fock pass over the rest of the Eq. 15 list fo
// (both built by pairs_merged_build)
void run_fock_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, const double *dc, double *F,
                   double *g_nuc, double *g_surf, int prec);
// screen with P (Eq. 18 bits into m18, Eq. 15 bits into m15) and build fg = the Eq. 18 list and
// fo = the Eq. 15 list without the Eq. 18 survivors, with FP64 header records; `dynamic` splits
// each at dp_thresh (Eq. 15 bound or Eq. 18 weight) into an FP64 part (fg, fo) and an FP32 part
// (fg_w, fo_w)
void pairs_merged_build(pcm_ctx *ctx, pcm_mol *mol, const double *P, bool dynamic);
// F += sum_k q_k L^k over the lists `strong` (FP64 records; FP32 Boys table when prec is mixed)
// and, for PCM_DYNAMIC, `weak` (FP32 records)
void run_fock_lists(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F, int prec, ListSel strong, ListSel weak);
// grow the V and primitive-block buffers for every class and tuning candidate of the Fock pass over ls
void fock_buffers(pcm_mol *mol, ListSel ls);
// contraction to F blocks and scatter of V sums held in vin (stride vnt), class cl of list pl
void fock_contract_scatter(pcm_ctx *ctx, pcm_mol *mol, const PairList &pl, int cl, const double *vin, int nch,
                           int vnt, const unsigned long long *memb, double *F);
void run_grad_batch(pcm_ctx *ctx, const std::vector<pcm_mol *> &mols, const std::vector<const double *> &P,
                    const std::vector<const double *> &q, const std::vector<double *> &g_nuc,
                    const std::vector<double *> &g_surf, int prec);
void surface_points(pcm_ctx *ctx, pcm_mol *mol, const double *r_explicit_dev);
// kind: PCM_PRECOND_RBJ (l = block size) or PCM_PRECOND_OCTREE (l = largest leaf)
void rbj_setup(pcm_ctx *ctx, pcm_mol *mol, int kind, int l, unsigned long long seed);
void rbj_prefetch(pcm_ctx *ctx, pcm_mol *mol);
void rbj_pending_drop(pcm_mol *mol);
SolveBatch *solve_batch_new(const std::vector<pcm_mol *> &mols);
void solve_batch_free(SolveBatch *b);
pcm_status solve_batch_run(pcm_ctx *ctx, SolveBatch &B, const std::vector<const double *> &v,
                           const std::vector<double *> &q, const pcm_solve_opts &o, pcm_solve_info *info);
// the batched FP64 solve as recorded launches for a captured graph (tables set up now), and the
// per-molecule report after a replay
// destroy a captured graph (if still alive): used when its batch or one of its molecules goes
void graph_drop(pcm_graph *g);
struct GraphSolveBufs;
GraphSolveBufs *graph_solve_bufs_new();
void graph_solve_bufs_free(GraphSolveBufs *b);
void solve_graph_launches(pcm_ctx *ctx, SolveBatch &B, const std::vector<const double *> &bz,
                          const std::vector<const double *> &c, const std::vector<double *> &q, double *E,
                          const pcm_solve_opts &o, int budget, GraphSolveBufs &gb, Launches &out);
void solve_graph_info(pcm_ctx *ctx, SolveBatch &B, double tol, pcm_solve_info *info, int *converged);
int host_rbj_partition(int M, const double *r, const double *zeta, int l, unsigned long long seed, int *perm,
                       int *blk_off);
int host_octree_partition(int M, const double *r, int leaf_max, int *perm, int *blk_off);
int block_partition(int kind, int M, const double *r, const double *zeta, int l, unsigned long long seed, int *perm,
                    int *blk_off);

inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }
// grid size for a bounds-checked 1-D launch over n items; never 0 (an empty molecule, e.g.
// with every surface point pruned, still launches one workgroup whose lanes all exit)
inline int grid_for(long long n, int block) { return n > 0 ? div_up(n, block) : 1; }
// grid of a grid-stride launch over n_items work items (one block per item up to 2^30 blocks)
inline int int_grid(long long n_items) { return (int)std::min<long long>(std::max<long long>(n_items, 1), 1 << 30); }
// copy a host descriptor table into the context's descriptor buffer (stream ordered)
inline void *upload_desc(pcm_ctx *ctx, const void *h, size_t bytes) {
    // at least 64 KiB, so that the small per-class tables of a call never move the buffer
    ctx->desc.ensure(std::max<size_t>(bytes, size_t(1) << 16));
    if (bytes) HIP_OK(hipMemcpyAsync(ctx->desc.p, h, bytes, hipMemcpyHostToDevice, ctx->stream));
    return ctx->desc.p;
}
