/*
 * pcm.h -- C ABI of the MI355X (gfx950) C-PCM / ISWIG solvation library.
 *
 * The library implements the solvation hot path of Liu, Luehr, Kulik and
 * Martinez, "Quantum Chemistry for Solvated Molecules on GPUs using Polarizable
 * Continuum Models" (arXiv:1505.07851):
 *   - the ISWIG surface (Sec. 2, Eqs. 3, 7, 9; parameters of Sec. 3),
 *   - the screened electrostatic integrals L^k_{mu nu} (Sec. 2, Eq. 6) used as
 *     c = L P (Eq. 5) and as the Fock correction sum_k q_k L^k (Eq. 10),
 *   - a matrix-free preconditioned CG solve of A q = -f (B z + c) (Eq. 1) with
 *     the dynamic threshold (Eq. 21) and randomized block-Jacobi preconditioner
 *     (Sec. 4b),
 *   - the energy (Eq. 13) and its gradient at fixed density (Eq. 14, Eq. 22).
 *
 * Conventions shared by every entry point:
 *   - atomic units (bohr, hartree, elementary charge);
 *   - FP64, row-major, contiguous arrays;
 *   - arrays documented as DEVICE are device pointers on the context's GPU
 *     (for example torch CUDA/HIP tensors); arrays documented as HOST are host
 *     memory read during the call and not retained;
 *   - the caller owns every numeric buffer; the library owns pcm_ctx and
 *     pcm_mol and the device workspace inside them; no call frees a caller
 *     buffer;
 *   - work is enqueued on the context's stream; pcm_esp, pcm_fock and pcm_grad
 *     are asynchronous with respect to the host, pcm_build_surface,
 *     pcm_update_geometry, pcm_solve and pcm_energy return after their results
 *     are complete;
 *   - every call returns a pcm_status; the message of the last failure is kept
 *     in the context (pcm_last_error); nothing throws or aborts across the ABI;
 *   - argument checks run before any GPU call, so PCM_E_ARG / PCM_E_UNSUPPORTED
 *     never leave partial device work behind;
 *   - one context per host thread.
 */
#ifndef PCM_H
#define PCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCM_OK = 0,
    PCM_E_ARG = 1,          /* invalid argument (null, non-finite, non-positive, out of range) */
    PCM_E_ALLOC = 2,        /* device or host allocation failed */
    PCM_E_HIP = 3,          /* a HIP runtime call failed (includes: no GPU present) */
    PCM_E_NOCONV = 4,       /* solver hit max_iter; q and info still hold the best iterate */
    PCM_E_NOTPD = 5,        /* a preconditioner block is not positive definite */
    PCM_E_UNSUPPORTED = 6,  /* angular momentum above d, or more than 8 primitives in a shell */
    PCM_E_STATE = 7         /* call made on an object in the wrong state (e.g. stale sizes) */
} pcm_status;

enum { PCM_FP64 = 0, PCM_MIXED = 1, PCM_DYNAMIC = 2 };
enum { PCM_PRECOND_NONE = 0, PCM_PRECOND_JACOBI = 1, PCM_PRECOND_RBJ = 2, PCM_PRECOND_OCTREE = 3 };

typedef struct pcm_ctx pcm_ctx;
typedef struct pcm_mol pcm_mol;
typedef struct pcm_batch pcm_batch;
typedef struct pcm_graph pcm_graph;

/* Model parameters (Sec. 2 and Sec. 3).
 *   eps            dielectric constant; f = (eps-1)/(eps+k_factor) (Eq. 1). Default 78.39.
 *   k_factor       k of Eq. 1; 0 (C-PCM) by default, 0.5 gives COSMO.
 *   zeta0          optimized exponent zeta of Eq. 7. Default 4.9.
 *   switch_thresh  points with switching value S_k below this are dropped (Sec. 3). Default 1e-8.
 *   schwarz_thresh primitive-pair screening cutoff (Eq. 15, Eq. 18). Default 1e-12.
 *   diag_const     constant of Eq. 3: A_kk = diag_const * zeta_k / S_k. Default sqrt(2/pi),
 *                  the r -> 0 limit of Eq. 2 for two equal Gaussians.
 *   precision      PCM_FP64, PCM_MIXED (FP32 Hermite/Boys evaluation with FP64 accumulation)
 *                  or PCM_DYNAMIC (per primitive pair: FP64 when its screening bound -- Eq. 18
 *                  for c and the gradient, Eq. 15 for F -- reaches dp_thresh, FP32 with FP64
 *                  accumulation otherwise; the per-pair precision choice of the paper's
 *                  ref. 51, applied to these one-electron integrals) for the integral
 *                  kernels. Default PCM_FP64.
 *   dp_thresh      PCM_DYNAMIC split threshold. Default 1e-6.
 *   autotune       1 (default): on first use of an integral kernel for a (class, precision,
 *                  size bucket) the library times a few pair/point chunk shapes and keeps the
 *                  fastest for the life of the context; results then depend on that choice
 *                  within rounding (chunk partial sums are added in a fixed order, so repeated
 *                  calls in one context are bitwise identical).  0: fixed shapes. */
typedef struct {
    double eps, k_factor, zeta0, switch_thresh, schwarz_thresh, diag_const;
    int precision;
    int autotune;
    double dp_thresh;
} pcm_params;

void pcm_default_params(pcm_params *p);

/* Contracted Cartesian Gaussian basis (Sec. 2, Eqs. 11-12).  HOST arrays.
 *   shell_atom[s]  atom carrying shell s (0..n_atoms-1)
 *   shell_l[s]     0, 1 or 2 (s, p, d); Cartesian components in lexicographic order
 *                  (x, y, z; xx, xy, xz, yy, yz, zz); basis functions numbered shell by shell
 *   shell_nprim[s] 1..8 primitives
 *   shell_off[s]   offset of the shell's primitives in prim_exp / prim_coef
 *   prim_exp, prim_coef  exponents (> 0) and raw contraction coefficients; the library
 *                  normalises every Cartesian component of every contracted shell to unit
 *                  self-overlap. */
typedef struct {
    int n_shells;
    const int *shell_atom, *shell_l, *shell_nprim, *shell_off;
    const double *prim_exp, *prim_coef;
} pcm_basis;

/* Solver options (Sec. 4b).
 *   precond     PCM_PRECOND_NONE, _JACOBI (diag(A)^-1), _RBJ (randomized block Jacobi) or
 *               _OCTREE (block Jacobi over the leaves of a spatial octree, the scheme RBJ is
 *               compared with in Sec. 4b-ii; see pcm_octree_partition)
 *   block       RBJ block size l (paper: 100), or the largest octree leaf (paper: 800);
 *               1..1024 for both
 *   seed        SplitMix64 seed of the RBJ partition (unused by the octree)
 *   tol         stop when ||A q - b||_2 < tol (Eq. 20), absolute, atomic units; use
 *               pcm_dynamic_threshold for the Eq. 21 schedule
 *   max_iter    bound on matrix-vector products
 *   warm_start  nonzero: q holds the initial guess on entry; zero: start from q = 0
 *   precision   PCM_FP64 (FP64 matvec) or PCM_MIXED (FP32 matvec inside FP64
 *               iterative refinement; FP64 residual, dots and energy)
 *   inner_rtol  relative residual reduction of each inner FP32 solve (mixed only; 0: 1e-4);
 *               an inner solve also stops after 400 iterations, and the outer FP64
 *               residual restarts it */
typedef struct {
    int precond;
    int block;
    unsigned long long seed;
    double tol;
    int max_iter;
    int warm_start;
    int precision;
    double inner_rtol;
} pcm_solve_opts;

void pcm_default_solve_opts(pcm_solve_opts *o);

/* Solver report (HOST struct filled by pcm_solve). */
typedef struct {
    int iters;          /* matrix-vector products with A (all precisions) */
    int refinements;    /* outer FP64 refinement steps (mixed) */
    double resid;       /* final ||A q - b||_2 recomputed in FP64 */
    double energy;      /* Eq. 13 energy at the returned q */
    double setup_ms;    /* preconditioner setup time */
    double solve_ms;    /* iteration time */
} pcm_solve_info;

/* Create a context bound to the current HIP device and `hip_stream` (a hipStream_t;
 * NULL = default stream).  `params` may be NULL for defaults.  No GPU call is made
 * here; device resources are created on first use.  Errors: PCM_E_ARG (null out,
 * non-finite or non-positive eps/zeta0, negative thresholds), PCM_E_ALLOC. */
pcm_status pcm_create(const pcm_params *params, void *hip_stream, pcm_ctx **out);
void pcm_destroy(pcm_ctx *ctx);
const char *pcm_last_error(const pcm_ctx *ctx);

/* Build the ISWIG surface and the screened pair lists (Sec. 2, Eqs. 3, 7, 9; Sec. 3;
 * Sec. 4a, Eq. 15).  HOST inputs: xyz[n_atoms*3], Z[n_atoms], radius[n_atoms] (cavity
 * radius in bohr, e.g. 1.2 x Bondi), sph_dirs[n_sph*3] unit vectors and sph_w[n_sph]
 * weights (sum 4 pi) of the unit-sphere rule, basis.  Point k = (atom I, sphere point j)
 * sits at R_I + radius_I u_j with exponent zeta0/(radius_I sqrt(w_j)); points with
 * S_k < switch_thresh are dropped; the kept points are ordered by atom, then j.  The
 * kept set and the Eq. 15 pair list are fixed for the life of the molecule (later
 * geometry updates do not re-prune), so energies stay smooth for differentiation.
 * Outputs: *out (owned by the library), *M_out = number of kept points.
 * Errors: PCM_E_ARG, PCM_E_UNSUPPORTED (l > 2 or nprim > 8), PCM_E_HIP, PCM_E_ALLOC. */
pcm_status pcm_build_surface(pcm_ctx *ctx, int n_atoms, const double *xyz, const double *Z, const double *radius,
                             int n_sph, const double *sph_dirs, const double *sph_w, const pcm_basis *basis,
                             pcm_mol **out, int *M_out);

/* Move nuclei (HOST xyz[n_atoms*3]) and, optionally, place surface points explicitly
 * (HOST r_surf[M*3], NULL = points follow their atoms).  Recomputes S_k, A_kk and the
 * pair geometry with the kept-point set and pair lists unchanged. */
pcm_status pcm_update_geometry(pcm_ctx *ctx, pcm_mol *mol, const double *xyz, const double *r_surf);

/* c_k = sum_{mu nu} P_{mu nu} L^k_{mu nu}, L^k = -(mu|erf(zeta_k|r-r_k|)/|r-r_k||nu)
 * (Sec. 2, Eqs. 5-6, 12).  Primitive pairs are screened with |P| times the Eq. 15 bound
 * (Eq. 18).  DEVICE: P[nbf*nbf] (symmetric), c[M] (written).  bz (DEVICE, may be NULL):
 * written with (B z)_k = sum_J Z_J erf(zeta_k |r_k-R_J|)/|r_k-R_J| (Eq. 4). */
pcm_status pcm_esp(pcm_ctx *ctx, pcm_mol *mol, const double *P, double *c, double *bz);

/* c (as pcm_esp) together with dc_k = d c_k / d r_k, the derivative of c_k with respect to the
 * position of its own surface point (Sec. 4c, Eq. 22: the operator-centre term gc of the
 * gradient, gc_k = q_k dc_k, reduced over primitive pairs like c).  One pass over the Eq. 18
 * list: the Hermite auxiliary values R^(0..L+1) of each (pair, point) evaluation give both the
 * potential and its derivative.  c equals pcm_esp's c to rounding (a different work split).
 * DEVICE: P[nbf*nbf], c[M] (written), bz[M] (may be NULL; Eq. 4), dc[M*3] (written), each
 * 8-byte aligned.  Errors: PCM_E_ARG (NULL or misaligned). */
pcm_status pcm_esp_deriv(pcm_ctx *ctx, pcm_mol *mol, const double *P, double *c, double *bz, double *dc);

/* F += sum_k q_k L^k (Eq. 10) and the Eq. 14 gradient (as pcm_fock followed by pcm_grad) with
 * one integral pass per primitive pair.  The Fock sums V_tuv = sum_k q_k R_tuv(k) (t+u+v <= L)
 * are the low orders of the V'_tuv (t+u+v <= L+1) that the basis-centre derivatives ga, gb of
 * Eq. 22 contract: the pairs of the Eq. 18 list for P accumulate V' once, for the gradient and,
 * where the Eq. 15 list holds them, for F; the Eq. 15 pairs outside the Eq. 18 list accumulate V
 * up to L for F alone.  F and the gradient equal pcm_fock's and pcm_grad's to rounding.  The
 * operator-centre term takes dc from pcm_esp_deriv, which must have been called with the same P
 * at the current geometry (not checked).  With PCM_DYNAMIC precision both lists are split at
 * dp_thresh by the larger of an entry's Eq. 15 bound and Eq. 18 weight.
 * DEVICE: P[nbf*nbf], q[M], dc[M*3], F[nbf*nbf] (accumulated), g_nuc[n_atoms*3] and
 * g_surf[M*3] (written; as pcm_grad), each 8-byte aligned.  Errors: PCM_E_ARG (NULL or
 * misaligned), PCM_E_UNSUPPORTED (a class needs more than 2^30 work items). */
pcm_status pcm_fock_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, const double *dc, double *F,
                         double *g_nuc, double *g_surf);

/* F_{mu nu} += sum_k q_k L^k_{mu nu} (Sec. 2, Eq. 10; Sec. 4a, Eqs. 16-17), over the Eq. 15
 * list; the full symmetric matrix is accumulated.  DEVICE: q[M], F[nbf*nbf] (in/out). */
pcm_status pcm_fock(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F);

/* Solve A q = -f v (Sec. 2, Eq. 1, with v = B z + c) by preconditioned CG (Sec. 4b).
 * DEVICE: v[M], q[M] (in: initial guess when opts->warm_start; out: solution).
 * HOST: opts (NULL = defaults), info (may be NULL).  Returns PCM_E_NOCONV when max_iter
 * is reached (q and info hold the last iterate), PCM_E_NOTPD when an RBJ block is not
 * positive definite. */
pcm_status pcm_solve(pcm_ctx *ctx, pcm_mol *mol, const double *v, const pcm_solve_opts *opts, double *q,
                     pcm_solve_info *info);

/* Energy of Eq. 13: (Bz)^T q + c^T q + 1/(2f) q^T A q, in FP64.  DEVICE: bz[M], c[M], q[M].
 * HOST: *E. */
pcm_status pcm_energy(pcm_ctx *ctx, pcm_mol *mol, const double *bz, const double *c, const double *q, double *E);

/* One rank's share of the product y = A x (Sec. 2, Eqs. 2-3, 8), the per-GPU work of the
 * sharded matvec: A is split into 256 x 256 tile pairs (I, J >= I) taken in the order
 * I = 0.., J = I..; rank r of nranks evaluates the pairs at positions p with p mod nranks = r
 * (each unordered point pair once, feeding both its row and its column) and adds A_kk x_k on
 * the rows of the diagonal tile pairs it owns.  Summing y over ranks 0 .. nranks-1 gives A x,
 * which is the reduce-scatter a multi-GPU solve would perform.  DEVICE: x[M], y[M] (written).
 * Errors: PCM_E_ARG (NULL, nranks < 1, rank outside [0, nranks)). */
pcm_status pcm_matvec_share(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks);

/* pcm_matvec_share with no allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and result bits as pcm_matvec_share; every intermediate (packed
 * points, tile boxes, a copy of x, the tile-pair list, the (nT x M) partial slots,
 * nT = ceil(M / 256)) lives in one fixed 64 MiB device array per GPU, held from library load
 * to process end, whose address is looked up when a context first uses the device.  That
 * bounds M to about 45,000 points.  The call only enqueues work on the context's stream (it
 * does not synchronise); y is complete when the stream reaches it.  Every call on one GPU
 * shares the array and overwrites what the previous call left there, so calls that can
 * overlap on one GPU (other streams, other contexts, other host threads) race: serialise
 * them.  DEVICE: x[M], y[M] (written), 8-byte aligned.  Errors (no GPU work is enqueued):
 * PCM_E_ARG (NULL, misaligned, rank outside [0, nranks), molecule of another context, or M
 * too large for the array), PCM_E_STATE (the context has not been used on a device yet, or
 * the current device is not the context's). */
pcm_status pcm_matvec_share_noalloc(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks);

/* Gradient of the Eq. 13 energy at fixed density (Sec. 2, Eq. 14; Sec. 4c, Eq. 22) for a
 * solved q.  Primitive pairs are screened as in pcm_esp (Eq. 18).  DEVICE: P[nbf*nbf],
 * q[M]; outputs g_nuc[n_atoms*3] (derivative with respect to nuclear positions with the
 * surface points held fixed: basis centres, B, and the switching functions inside A_kk)
 * and g_surf[M*3] (derivative with respect to each surface point).  Points move with
 * their atom, so the total nuclear gradient is g_nuc[I] + sum_{k on I} g_surf[k]. */
pcm_status pcm_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, double *g_nuc, double *g_surf);

/* Dynamic CG threshold (Sec. 4b-i, Eq. 21): the delta whose predicted energy error
 * 0.01 delta^1.07 equals 1e-3 times the previous DIIS error, clamped to [1e-10, 1];
 * 1.0 when diis_err_prev < 0 (first SCF step).  Pure host function. */
double pcm_dynamic_threshold(double diis_err_prev);

/* CG threshold policies of Sec. 4b-i, one call per SCF step with the previous step's DIIS
 * error (max element of X^T (SPF - FPS) X; negative on the first step).  Pure host functions.
 *   PCM_THRESH_FIXED      delta every step
 *   PCM_THRESH_TWO_DELTA  2-delta switching: the loose delta_1 = scale * delta until the DIIS
 *                         error has reached switch_at, the tight delta_2 = delta from then on
 *                         (the switch happens once: `switched` latches; paper: scale 1e4,
 *                         switch_at 1e-3, delta 1e-5..1e-7)
 *   PCM_THRESH_DYNAMIC    pcm_dynamic_threshold (Eq. 21); delta, scale, switch_at unused
 * pcm_default_threshold_policy fills delta 1e-6, scale 1e4, switch_at 1e-3, switched 0.
 * pcm_cg_threshold returns the threshold for this step (and updates `switched`), or -1 on a
 * bad policy (NULL, unknown kind, non-finite or non-positive delta, scale < 1, switch_at < 0). */
enum { PCM_THRESH_FIXED = 0, PCM_THRESH_TWO_DELTA = 1, PCM_THRESH_DYNAMIC = 2 };
typedef struct {
    int kind;
    double delta;
    double scale;
    double switch_at;
    int switched;
} pcm_threshold_policy;
void pcm_default_threshold_policy(pcm_threshold_policy *p, int kind);
double pcm_cg_threshold(pcm_threshold_policy *p, double diis_err_prev);

/* Randomized block-Jacobi partition (Sec. 4b-ii) of M points, on the host: a SplitMix64
 * stream from `seed` picks a random pivot among the unassigned points (kept in ascending
 * order; index floor(u n_left), u = (x >> 11) 2^-53); the block is the pivot plus the l-1
 * unassigned points with the largest |A_kl| (ties: smaller index first); members are
 * stored ascending; repeated until every point is assigned.  HOST: r[M*3], zeta[M];
 * outputs perm[M] and blk_off[n_blocks+1] (capacity M+1); returns n_blocks, or -1 on a
 * bad argument. */
int pcm_rbj_partition(int M, const double *r, const double *zeta, int l, unsigned long long seed, int *perm,
                      int *blk_off);

/* Spatial octree partition (the block-Jacobi scheme of Sec. 4b-ii that RBJ is compared
 * with), on the host.  The root is the cube centred on the midpoint of the points' bounding
 * box with half-side half its largest extent; a cell with more than leaf_max points is cut
 * into octants at its centre (octant = [x >= cx] + 2 [y >= cy] + 4 [z >= cz]); leaves are
 * emitted depth first in octant order, empty cells dropped, members ascending; a cell still
 * too full at depth 40 (coincident points) is cut into consecutive runs of leaf_max.
 * HOST: r[M*3]; outputs perm[M] and blk_off[n_blocks+1] (capacity M+1); returns
 * n_blocks, or -1 on a bad argument (M < 1, leaf_max < 1, NULL, non-finite r). */
int pcm_octree_partition(int M, const double *r, int leaf_max, int *perm, int *blk_off);

/* Copy the surface out.  DEVICE outputs (any may be NULL): r[M*3], zeta[M], S[M],
 * Akk[M], owner[M] (int32 atom index), sph[M] (int32 sphere-point index). */
pcm_status pcm_surface_get(pcm_ctx *ctx, const pcm_mol *mol, double *r, double *zeta, double *S, double *Akk,
                           int *owner, int *sph);

/* Sizes.  HOST outputs (any may be NULL): M, nbf, n_atoms; pairs_fock[6] and
 * pairs_esp[6] = surviving primitive pairs per class (ss, sp, sd, pp, pd, dd) of the
 * Eq. 15 list and of the last Eq. 18 list built by pcm_esp / pcm_grad; sp_fock[6] and
 * sp_esp[6] = surviving shell pairs per class. */
pcm_status pcm_mol_sizes(const pcm_mol *mol, int *M, int *nbf, int *n_atoms, long long *pairs_fock,
                         long long *pairs_esp, long long *sp_fock, long long *sp_esp);

/* Copy a screened primitive-pair list out (HOST arrays of capacity sum(pairs_*)):
 * list 0 = Eq. 15 (Fock) list, 1 = last Eq. 18 list; entries in the order class, shell
 * pair (a, b) with l_a <= l_b (a <= b for equal l), primitive i of a, j of b. */
pcm_status pcm_pair_list(pcm_ctx *ctx, const pcm_mol *mol, int which, int *cls, int *a, int *b, int *i, int *j);

void pcm_mol_destroy(pcm_mol *mol);

/* Batches: several molecules (e.g. conformers with uneven surface sizes) whose kernels run
 * as one launch over a shared table of work items, with per-molecule scalars, iteration
 * counters and convergence flags kept on the device.  pcm_batch_create records the HOST
 * array mols[n] (n >= 1, distinct molecules built on ctx); the batch holds no reference
 * count, so destroy it before any of its molecules.  Errors: PCM_E_ARG. */
pcm_status pcm_batch_create(pcm_ctx *ctx, pcm_mol *const *mols, int n, pcm_batch **out);
void pcm_batch_destroy(pcm_batch *batch);

/* pcm_esp for every molecule of the batch (Sec. 2, Eqs. 5-6, 12, 18): the density-screened
 * pair lists are built per molecule, then one launch per angular class evaluates every
 * molecule's pairs against its points.  HOST arrays of DEVICE pointers P[n] (nbf_i^2),
 * c[n] (M_i, written); bz may be NULL, or hold DEVICE pointers (NULL entries skipped).
 * Molecule i gets bitwise the c of pcm_esp on the same context. */
pcm_status pcm_esp_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *P, double *const *c,
                           double *const *bz);

/* pcm_fock for every molecule of the batch (Sec. 2, Eq. 10; Sec. 4a, Eqs. 16-17): one launch
 * per angular class for the point sums, then per-molecule contraction into F.  HOST arrays
 * of DEVICE pointers q[n] (M_i), F[n] (nbf_i^2, accumulated). */
pcm_status pcm_fock_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *q, double *const *F);

/* pcm_solve for every molecule of the batch at once (Sec. 2, Eq. 1; Sec. 4b).  HOST arrays
 * of DEVICE pointers v[n] and q[n] (molecule i: v[i][M_i], q[i][M_i]); HOST info[n] (may be
 * NULL).  Groups of PCG iterations are replayed from a captured hipGraph; molecules that
 * have converged skip the remaining work of their group, so every molecule receives the
 * iterates it would get alone.  PCM_E_NOCONV when any molecule reached max_iter. */
pcm_status pcm_solve_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *v, const pcm_solve_opts *opts,
                             double *const *q, pcm_solve_info *info);

/* pcm_grad for every molecule of the batch (Sec. 2, Eq. 14; Sec. 4c, Eq. 22): per angular
 * class one launch of the point side and one of the pair side over all molecules, then
 * per-molecule contraction and the per-point and per-atom sums.  Each molecule's work split
 * does not depend on the others, so the results equal those of pcm_grad bit for bit.  HOST
 * arrays of DEVICE pointers P[n] (nbf_i^2), q[n] (M_i), g_nuc[n] (n_atoms_i*3, written),
 * g_surf[n] (M_i*3, written).  Errors: PCM_E_ARG (NULL array or entry), PCM_E_UNSUPPORTED
 * (one class of the batch needs more than 2^30 work items). */
pcm_status pcm_grad_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *P, const double *const *q,
                            double *const *g_nuc, double *const *g_surf);

/* One solvation pass of every molecule of a batch captured as a single hipGraph (many conformers
 * with uneven surfaces in one launch): for molecule i, the Eq. 18 list screened with P[i] at
 * capture and its density coefficients rebuilt from the current contents of P[i] at every replay,
 * c[i] = L P[i] (Sec. 2, Eqs. 5-6) and bz[i] (Eq. 4), the preconditioned CG solve of
 * A q = -f (bz + c) (Eq. 1, Sec. 4b) in FP64 from q = 0 with a fixed budget of opts->max_iter
 * iterations (a molecule stops on the device once ||r|| < opts->tol on the CG recurrence; its
 * remaining iterations skip), the explicit residual, q[i], the Eq. 13 energy E[i], and
 * F[i] += L^T q[i] (Eq. 10).  Capture does all host work (screening, chunk choice and tuning,
 * descriptor and solver tables, the block-Jacobi partition and inverses); a replay launches
 * kernels only and allocates nothing.  The arrays are bound by address: HOST arrays of DEVICE
 * pointers P[n] (nbf_i^2, read at each replay), c[n], bz[n], q[n] (M_i, written), F[n]
 * (nbf_i^2, accumulated at each replay); DEVICE E[n] (written).  opts: NULL = defaults; precond,
 * block, seed and tol as for pcm_solve, max_iter is the iteration budget (1..100000), precision
 * must be PCM_FP64.  The pair lists stay as screened at capture: capture again (after
 * pcm_graph_destroy) when the densities change enough to change the Eq. 18 screening.
 * While the graph exists its batch and molecules refuse every call that could move their buffers
 * (PCM_E_STATE); destroy the graph before the batch, the molecules or the context.
 * Errors: PCM_E_ARG, PCM_E_UNSUPPORTED (precision other than FP64), PCM_E_STATE (batch or a
 * molecule already bound), PCM_E_HIP, PCM_E_ALLOC. */
pcm_status pcm_graph_capture(pcm_ctx *ctx, pcm_batch *batch, const double *const *P, double *const *c,
                             double *const *bz, double *const *q, double *const *F, double *E,
                             const pcm_solve_opts *opts, pcm_graph **out);
/* Replay the captured pass on the context's stream (asynchronous; one hipGraphLaunch). */
pcm_status pcm_graph_launch(pcm_ctx *ctx, pcm_graph *g);
/* After a replay (synchronises the stream): HOST info[n] (may be NULL) with iters (CG iterations),
 * resid (explicit ||A q - b||_2) and energy of each molecule; HOST *nodes (may be NULL) = kernel
 * nodes in the graph.  Returns PCM_E_NOCONV when a molecule's explicit residual is not below tol
 * (the budget ran out, or the recurrence converged ahead of the explicit residual: the captured
 * solve has no restarts). */
pcm_status pcm_graph_info(pcm_ctx *ctx, pcm_graph *g, pcm_solve_info *info, long long *nodes);
void pcm_graph_destroy(pcm_graph *g);

/* Per-kernel timing.  pcm_profile_enable(ctx, 1) clears previous records and makes every
 * heavy launch (integral, matvec, gradient and preconditioner kernels) record a pair of HIP
 * events on the context's stream; pcm_profile_collect synchronises the stream, aggregates
 * the records by kernel name and returns the number of names (-1 on error);
 * pcm_profile_entry(i) reports name (HOST buffer of name_cap bytes), total milliseconds,
 * number of launches and work units (pair x point evaluations for integral kernels,
 * unordered point pairs for the matvec, inverse-block elements for the preconditioner).  Profiling adds two event records per
 * launch and is off by default. */
pcm_status pcm_profile_enable(pcm_ctx *ctx, int on);
int pcm_profile_collect(pcm_ctx *ctx);
pcm_status pcm_profile_entry(const pcm_ctx *ctx, int i, char *name, int name_cap, double *ms, long long *launches,
                             double *work);

#ifdef __cplusplus
}
#endif
#endif /* PCM_H */
