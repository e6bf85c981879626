// C ABI of the gfx950 C-PCM library (declared in include/pcm.h).  Argument validation runs
// on the host before any HIP call; every failure is reported as a pcm_status with a message
// kept in the context.
#include "pcm_internal.h"

#include <algorithm>
#include <iterator>
#include <cstring>
#include <new>

namespace {

bool is_fin(double x) { return std::isfinite(x); }

// device arrays of FP64 (and int32 pairs) must be 8-byte aligned; NULL counts as aligned
bool misaligned(const void *p) { return ((uintptr_t)p & 7) != 0; }
template <typename... A> bool any_misaligned(const A *...p) { return (misaligned(p) || ...); }

template <typename T> void upload(pcm_ctx *ctx, DevBuf<T> &d, const T *h, size_t n) {
    d.ensure(n ? n : 1);
    if (n) HIP_OK(hipMemcpyAsync(d.p, h, n * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
}

void release_list(PairList &pl) {
    pl.spo.release(); pl.cnt.release(); pl.mask.release();
    pl.ent_sp.release(); pl.ent_ij.release(); pl.rec.release(); pl.vperm.release();
}

void release_mol(pcm_mol *m) {
    rbj_pending_drop(m);
    DevBuf<double> *dbl[] = {&m->xyz, &m->Z, &m->rad, &m->dirs, &m->w, &m->pexp, &m->pcoef, &m->cn, &m->px, &m->py,
                             &m->pz, &m->zeta, &m->S, &m->Akk, &m->qpad, &m->part, &m->vbuf, &m->r_surf_buf,
                             &m->fprim, &m->gpair, &m->gsp, &m->sv, &m->rbj_inv};
    for (auto *b : dbl) b->release();
    DevBuf<int> *ints[] = {&m->sl, &m->snp, &m->soff, &m->satom, &m->bfo, &m->cnoff, &m->keep, &m->spa, &m->spb,
                           &m->atom_sp_off_a, &m->atom_sp_a, &m->atom_sp_off_b, &m->atom_sp_b, &m->scan_tmp,
                           &m->rbj_perm, &m->rbj_off};
    for (auto *b : ints) b->release();
    m->rbj_ioff.release();
    m->pti64.release();
    m->pti32.release();
    if (m->solo) solve_batch_free(m->solo);
    m->solo = nullptr;
    release_list(m->fock);
    release_list(m->esp);
    release_list(m->fock_w);
    release_list(m->esp_w);
    release_list(m->fg);
    release_list(m->fg_w);
    release_list(m->fo);
    release_list(m->fo_w);
    m->m15.release();
    m->mtmp.release();
    m->ctmp.release();
    m->pperm.release();
    m->okey.release();
    m->oval.release();
    m->osort.release();
    m->m18.release();
    m->c18.release();
}

// candidate shell pairs, classes concatenated; (a, b) with l_a <= l_b (a <= b for equal l)
void build_candidates(pcm_mol *m) {
    std::vector<int> by_l[3];
    for (int s = 0; s < m->ns; ++s) by_l[m->h_sl[s]].push_back(s);
    m->h_spa.clear();
    m->h_spb.clear();
    for (int c = 0; c < NCLS; ++c) {
        m->sp_cls_off[c] = (long long)m->h_spa.size();
        const auto &A = by_l[CLS_LA[c]], &B = by_l[CLS_LB[c]];
        for (int a : A)
            for (int b : B) {
                if (CLS_LA[c] == CLS_LB[c] && b < a) continue;
                m->h_spa.push_back(a);
                m->h_spb.push_back(b);
            }
    }
    m->sp_cls_off[NCLS] = (long long)m->h_spa.size();
}

void build_atom_lists(pcm_ctx *ctx, pcm_mol *m) {
    long long nsp = m->sp_cls_off[NCLS];
    std::vector<int> ca(m->N + 1, 0), cb(m->N + 1, 0);
    for (long long s = 0; s < nsp; ++s) {
        ++ca[m->h_satom[m->h_spa[s]] + 1];
        ++cb[m->h_satom[m->h_spb[s]] + 1];
    }
    for (int i = 0; i < m->N; ++i) {
        ca[i + 1] += ca[i];
        cb[i + 1] += cb[i];
    }
    std::vector<int> la(nsp), lb(nsp), fa(ca.begin(), ca.end() - 1), fb(cb.begin(), cb.end() - 1);
    for (long long s = 0; s < nsp; ++s) {
        la[fa[m->h_satom[m->h_spa[s]]]++] = (int)s;
        lb[fb[m->h_satom[m->h_spb[s]]]++] = (int)s;
    }
    upload(ctx, m->atom_sp_off_a, ca.data(), ca.size());
    upload(ctx, m->atom_sp_off_b, cb.data(), cb.size());
    upload(ctx, m->atom_sp_a, la.data(), la.size());
    upload(ctx, m->atom_sp_b, lb.data(), lb.size());
}

pcm_status check_basis(pcm_ctx *ctx, int n_atoms, const pcm_basis *b, int *nprim_total) {
    if (!b) return fail(ctx, PCM_E_ARG, "basis is NULL");
    if (b->n_shells < 0) return fail(ctx, PCM_E_ARG, "n_shells < 0");
    *nprim_total = 0;
    if (b->n_shells == 0) return PCM_OK;
    if (!b->shell_atom || !b->shell_l || !b->shell_nprim || !b->shell_off || !b->prim_exp || !b->prim_coef)
        return fail(ctx, PCM_E_ARG, "basis array is NULL");
    long long np = 0;
    for (int s = 0; s < b->n_shells; ++s) {
        int l = b->shell_l[s], n = b->shell_nprim[s];
        if (l < 0) return fail(ctx, PCM_E_ARG, "negative angular momentum in shell " + std::to_string(s));
        if (l > 2) return fail(ctx, PCM_E_UNSUPPORTED, "angular momentum above d in shell " + std::to_string(s));
        if (n < 1) return fail(ctx, PCM_E_ARG, "shell " + std::to_string(s) + " has no primitives");
        if (n > 8) return fail(ctx, PCM_E_UNSUPPORTED, "more than 8 primitives in shell " + std::to_string(s));
        if (b->shell_atom[s] < 0 || b->shell_atom[s] >= n_atoms)
            return fail(ctx, PCM_E_ARG, "shell_atom out of range in shell " + std::to_string(s));
        if (b->shell_off[s] < 0) return fail(ctx, PCM_E_ARG, "negative shell_off");
        np = std::max<long long>(np, (long long)b->shell_off[s] + n);
    }
    if (np > (1LL << 30)) return fail(ctx, PCM_E_ARG, "too many primitives");
    for (int s = 0; s < b->n_shells; ++s)
        for (int i = 0; i < b->shell_nprim[s]; ++i) {
            double e = b->prim_exp[b->shell_off[s] + i], c = b->prim_coef[b->shell_off[s] + i];
            if (!is_fin(e) || !(e > 0.0)) return fail(ctx, PCM_E_ARG, "non-positive or non-finite exponent");
            if (!is_fin(c)) return fail(ctx, PCM_E_ARG, "non-finite contraction coefficient");
        }
    *nprim_total = (int)np;
    return PCM_OK;
}

}  // namespace

pcm_status check_solve_opts(pcm_ctx *ctx, const pcm_solve_opts *opts, pcm_solve_opts &o) {
    pcm_default_solve_opts(&o);
    if (opts) o = *opts;
    if (o.precond < PCM_PRECOND_NONE || o.precond > PCM_PRECOND_OCTREE) return fail(ctx, PCM_E_ARG, "bad precond");
    if ((o.precond == PCM_PRECOND_RBJ || o.precond == PCM_PRECOND_OCTREE) && (o.block < 1 || o.block > 1024))
        return fail(ctx, PCM_E_ARG, "block-Jacobi block size must be in [1, 1024]");
    if (!is_fin(o.tol) || !(o.tol > 0.0)) return fail(ctx, PCM_E_ARG, "tol must be > 0");
    if (o.max_iter < 1) return fail(ctx, PCM_E_ARG, "max_iter must be >= 1");
    if (o.precision != PCM_FP64 && o.precision != PCM_MIXED) return fail(ctx, PCM_E_ARG, "bad precision");
    if (!is_fin(o.inner_rtol) || o.inner_rtol < 0.0 || o.inner_rtol >= 1.0)
        return fail(ctx, PCM_E_ARG, "inner_rtol must be in [0, 1)");
    return PCM_OK;
}

namespace {

// Pair records are FP64 in the FP64 and mixed forms (the mixed kernels interpolate the Boys
// function in FP32 but read FP64 pair data); with PCM_DYNAMIC the weak lists hold FP32 records
// (pairs_prepare_* take PCM_MIXED to mean FP32 records).
static void lists_geometry(pcm_ctx *ctx, pcm_mol *mol) {
    pairs_prepare_geometry(ctx, mol, mol->fock, PCM_FP64);
    if (ctx->prm.precision == PCM_DYNAMIC) pairs_prepare_geometry(ctx, mol, mol->fock_w, PCM_MIXED);
}

}  // namespace

pcm_status density_list(pcm_ctx *ctx, pcm_mol *mol, const double *P) {
    pairs_build(ctx, mol, mol->esp, P, 1);
    if (ctx->prm.precision == PCM_DYNAMIC) {
        pairs_split(ctx, mol, mol->esp, mol->esp_w, P, ctx->prm.dp_thresh);
        pairs_prepare_density(ctx, mol, mol->esp, P, PCM_FP64);
        pairs_prepare_density(ctx, mol, mol->esp_w, P, PCM_MIXED);
    } else {
        pairs_prepare_density(ctx, mol, mol->esp, P, PCM_FP64);
    }
    mol->esp_valid = true;
    return PCM_OK;
}

extern "C" {

void pcm_default_params(pcm_params *p) {
    if (!p) return;
    p->eps = 78.39;
    p->k_factor = 0.0;
    p->zeta0 = 4.9;
    p->switch_thresh = 1e-8;
    p->schwarz_thresh = 1e-12;
    p->diag_const = std::sqrt(2.0 / M_PI);
    p->precision = PCM_FP64;
    p->autotune = 1;
    p->dp_thresh = 1e-6;
}

void pcm_default_solve_opts(pcm_solve_opts *o) {
    if (!o) return;
    o->precond = PCM_PRECOND_JACOBI;
    o->block = 100;
    o->seed = 0;
    o->tol = 1e-6;
    o->max_iter = 10000;
    o->warm_start = 0;
    o->precision = PCM_FP64;
    o->inner_rtol = 1e-4;
}

pcm_status pcm_create(const pcm_params *params, void *hip_stream, pcm_ctx **out) {
    if (!out) return PCM_E_ARG;
    *out = nullptr;
    pcm_params p;
    pcm_default_params(&p);
    if (params) p = *params;
    if (!is_fin(p.eps) || !(p.eps > 1.0) || !is_fin(p.k_factor) || p.k_factor < 0.0 || !is_fin(p.zeta0) ||
        !(p.zeta0 > 0.0) || !is_fin(p.switch_thresh) || p.switch_thresh < 0.0 || !is_fin(p.schwarz_thresh) ||
        p.schwarz_thresh < 0.0 || !is_fin(p.diag_const) || !(p.diag_const > 0.0) ||
        (p.precision != PCM_FP64 && p.precision != PCM_MIXED && p.precision != PCM_DYNAMIC) ||
        (p.autotune != 0 && p.autotune != 1) || !is_fin(p.dp_thresh) || p.dp_thresh < 0.0)
        return PCM_E_ARG;
    pcm_ctx *c = new (std::nothrow) pcm_ctx();
    if (!c) return PCM_E_ALLOC;
    c->prm = p;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return PCM_OK;
}

void pcm_destroy(pcm_ctx *ctx) {
    if (!ctx) return;
    ctx->boys64.release();
    ctx->boys32.release();
    ctx->scal.release();
    ctx->iscal.release();
    ctx->lscal.release();
    delete ctx;
}

const char *pcm_last_error(const pcm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pcm_status pcm_build_surface(pcm_ctx *ctx, int n_atoms, const double *xyz, const double *Z, const double *radius,
                             int n_sph, const double *sph_dirs, const double *sph_w, const pcm_basis *basis,
                             pcm_mol **out, int *M_out) {
    if (!ctx) return PCM_E_ARG;
    if (!xyz || !Z || !radius || !sph_dirs || !sph_w || !out || !M_out) return fail(ctx, PCM_E_ARG, "NULL argument");
    *out = nullptr;
    *M_out = 0;
    if (n_atoms < 1 || n_sph < 1) return fail(ctx, PCM_E_ARG, "n_atoms and n_sph must be positive");
    if ((long long)n_atoms * n_sph > (1LL << 30)) return fail(ctx, PCM_E_ARG, "too many raw surface points");
    for (int i = 0; i < 3 * n_atoms; ++i)
        if (!is_fin(xyz[i])) return fail(ctx, PCM_E_ARG, "non-finite coordinate");
    for (int i = 0; i < n_atoms; ++i) {
        if (!is_fin(Z[i]) || Z[i] < 0.0) return fail(ctx, PCM_E_ARG, "nuclear charge must be finite and >= 0");
        if (!is_fin(radius[i]) || !(radius[i] > 0.0)) return fail(ctx, PCM_E_ARG, "radius must be finite and > 0");
    }
    for (int j = 0; j < n_sph; ++j) {
        if (!is_fin(sph_dirs[3 * j]) || !is_fin(sph_dirs[3 * j + 1]) || !is_fin(sph_dirs[3 * j + 2]))
            return fail(ctx, PCM_E_ARG, "non-finite sphere direction");
        if (!is_fin(sph_w[j]) || !(sph_w[j] > 0.0)) return fail(ctx, PCM_E_ARG, "sphere weight must be > 0");
    }
    int np = 0;
    pcm_status st = check_basis(ctx, n_atoms, basis, &np);
    if (st != PCM_OK) return st;
    pcm_mol *m = new (std::nothrow) pcm_mol();
    if (!m) return fail(ctx, PCM_E_ALLOC, "host allocation failed");
    m->owner_ctx = ctx;
    st = guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        m->N = n_atoms;
        m->nsph = n_sph;
        m->zeta0 = ctx->prm.zeta0;
        m->h_xyz.assign(xyz, xyz + 3 * n_atoms);
        m->h_Z.assign(Z, Z + n_atoms);
        m->h_rad.assign(radius, radius + n_atoms);
        m->h_dirs.assign(sph_dirs, sph_dirs + 3 * n_sph);
        m->h_w.assign(sph_w, sph_w + n_sph);
        m->ns = basis->n_shells;
        m->nprim = np;
        m->h_sl.assign(basis->shell_l, basis->shell_l + m->ns);
        m->h_snp.assign(basis->shell_nprim, basis->shell_nprim + m->ns);
        m->h_soff.assign(basis->shell_off, basis->shell_off + m->ns);
        m->h_satom.assign(basis->shell_atom, basis->shell_atom + m->ns);
        m->h_pexp.assign(basis->prim_exp, basis->prim_exp + np);
        m->h_pcoef.assign(basis->prim_coef, basis->prim_coef + np);
        m->h_bf.resize(m->ns);
        m->h_cnoff.resize(m->ns);
        int bf = 0, cno = 0;
        for (int s = 0; s < m->ns; ++s) {
            m->h_bf[s] = bf;
            m->h_cnoff[s] = cno;
            bf += ncart(m->h_sl[s]);
            cno += ncart(m->h_sl[s]) * m->h_snp[s];
        }
        m->nbf = bf;
        upload(ctx, m->xyz, m->h_xyz.data(), m->h_xyz.size());
        upload(ctx, m->Z, m->h_Z.data(), m->h_Z.size());
        upload(ctx, m->rad, m->h_rad.data(), m->h_rad.size());
        upload(ctx, m->dirs, m->h_dirs.data(), m->h_dirs.size());
        upload(ctx, m->w, m->h_w.data(), m->h_w.size());
        upload(ctx, m->sl, m->h_sl.data(), m->h_sl.size());
        upload(ctx, m->snp, m->h_snp.data(), m->h_snp.size());
        upload(ctx, m->soff, m->h_soff.data(), m->h_soff.size());
        upload(ctx, m->satom, m->h_satom.data(), m->h_satom.size());
        upload(ctx, m->bfo, m->h_bf.data(), m->h_bf.size());
        upload(ctx, m->cnoff, m->h_cnoff.data(), m->h_cnoff.size());
        upload(ctx, m->pexp, m->h_pexp.data(), m->h_pexp.size());
        upload(ctx, m->pcoef, m->h_pcoef.data(), m->h_pcoef.size());
        m->cn.ensure(cno ? cno : 1);
        if (m->ns) basis_normalise(ctx, m);
        surface_build(ctx, m, true);
        surface_points(ctx, m, nullptr);
        build_candidates(m);
        upload(ctx, m->spa, m->h_spa.data(), m->h_spa.size());
        upload(ctx, m->spb, m->h_spb.data(), m->h_spb.size());
        build_atom_lists(ctx, m);
        pairs_build(ctx, m, m->fock, nullptr, 0);
        if (ctx->prm.precision == PCM_DYNAMIC) pairs_split(ctx, m, m->fock, m->fock_w, nullptr, ctx->prm.dp_thresh);
        lists_geometry(ctx, m);
        HIP_OK(hipStreamSynchronize(ctx->stream));
        return PCM_OK;
    });
    if (st != PCM_OK) {
        release_mol(m);
        delete m;
        return st;
    }
    *out = m;
    *M_out = m->M;
    return PCM_OK;
}

pcm_status pcm_update_geometry(pcm_ctx *ctx, pcm_mol *mol, const double *xyz, const double *r_surf) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !xyz) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    for (int i = 0; i < 3 * mol->N; ++i)
        if (!is_fin(xyz[i])) return fail(ctx, PCM_E_ARG, "non-finite coordinate");
    if (r_surf)
        for (long long i = 0; i < 3LL * mol->M; ++i)
            if (!is_fin(r_surf[i])) return fail(ctx, PCM_E_ARG, "non-finite surface coordinate");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        mol->h_xyz.assign(xyz, xyz + 3 * mol->N);
        upload(ctx, mol->xyz, mol->h_xyz.data(), mol->h_xyz.size());
        // explicit points go through a buffer the molecule keeps (sized once, reused by later calls)
        if (r_surf) upload(ctx, mol->r_surf_buf, r_surf, 3 * (size_t)mol->M);
        surface_points(ctx, mol, r_surf ? mol->r_surf_buf.p : nullptr);
        lists_geometry(ctx, mol);
        HIP_OK(hipStreamSynchronize(ctx->stream));
        mol->esp_valid = false;
        mol->rbj_valid = false;
        rbj_prefetch(ctx, mol);
        return PCM_OK;
    });
}


pcm_status pcm_esp(pcm_ctx *ctx, pcm_mol *mol, const double *P, double *c, double *bz) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !P || !c) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(P, c, bz)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        density_list(ctx, mol, P);
        run_esp(ctx, mol, c, ctx->prm.precision);
        if (bz) run_bz(ctx, mol, bz);
        return PCM_OK;
    });
}

pcm_status pcm_esp_deriv(pcm_ctx *ctx, pcm_mol *mol, const double *P, double *c, double *bz, double *dc) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !P || !c || !dc) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(P, c, bz, dc))
        return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        density_list(ctx, mol, P);
        run_esp_deriv(ctx, mol, c, dc, ctx->prm.precision);
        if (bz) run_bz(ctx, mol, bz);
        return PCM_OK;
    });
}

pcm_status pcm_fock_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, const double *dc, double *F,
                         double *g_nuc, double *g_surf) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !P || !q || !dc || !F || !g_nuc || !g_surf) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(P, q, dc, F, g_nuc, g_surf))
        return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        const int prec = ctx->prm.precision;
        pairs_merged_build(ctx, mol, P, prec == PCM_DYNAMIC);
        run_fock_grad(ctx, mol, P, q, dc, F, g_nuc, g_surf, prec);
        return PCM_OK;
    });
}

pcm_status pcm_fock(pcm_ctx *ctx, pcm_mol *mol, const double *q, double *F) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !q || !F) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(q, F)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        run_fock(ctx, mol, q, F, ctx->prm.precision);
        return PCM_OK;
    });
}

pcm_status pcm_solve(pcm_ctx *ctx, pcm_mol *mol, const double *v, const pcm_solve_opts *opts, double *q,
                     pcm_solve_info *info) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !v || !q) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(v, q)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    pcm_solve_opts o;
    pcm_status vs = check_solve_opts(ctx, opts, o);
    if (vs != PCM_OK) return vs;
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        pcm_status st = run_solve(ctx, mol, v, o, q, info);
        if (st == PCM_E_NOCONV) ctx->err = "max_iter reached before the residual threshold";
        return st;
    });
}

pcm_status pcm_energy(pcm_ctx *ctx, pcm_mol *mol, const double *bz, const double *c, const double *q, double *E) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !bz || !c || !q || !E) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(bz, c, q)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        *E = run_energy(ctx, mol, bz, c, q);
        return PCM_OK;
    });
}

pcm_status pcm_matvec_share(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !x || !y) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(x, y)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (nranks < 1 || rank < 0 || rank >= nranks) return fail(ctx, PCM_E_ARG, "rank outside [0, nranks)");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        run_matvec_share(ctx, mol, x, y, rank, nranks);
        HIP_OK(hipStreamSynchronize(ctx->stream));
        return PCM_OK;
    });
}

pcm_status pcm_matvec_share_noalloc(pcm_ctx *ctx, pcm_mol *mol, const double *x, double *y, int rank, int nranks) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !x || !y) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(x, y)) return fail(ctx, PCM_E_ARG, "x and y must be 8-byte aligned");
    if (nranks < 1 || rank < 0 || rank >= nranks) return fail(ctx, PCM_E_ARG, "rank outside [0, nranks)");
    if (mol->owner_ctx != ctx) return fail(ctx, PCM_E_ARG, "molecule built on another context");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    if (!ctx->dev_ready) return fail(ctx, PCM_E_STATE, "context has not been used on a device yet");
    return guarded(ctx, [&]() -> pcm_status {
        int dev = -1;
        HIP_OK(hipGetDevice(&dev));
        if (dev != ctx->device) throw PcmError{PCM_E_STATE, "current device is not the context's device"};
        run_matvec_share_noalloc(ctx, mol, x, y, rank, nranks);
        return PCM_OK;
    });
}

pcm_status pcm_grad(pcm_ctx *ctx, pcm_mol *mol, const double *P, const double *q, double *g_nuc, double *g_surf) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !P || !q || !g_nuc || !g_surf) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (any_misaligned(P, q, g_nuc, g_surf)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (mol->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        density_list(ctx, mol, P);
        run_grad(ctx, mol, P, q, g_nuc, g_surf, ctx->prm.precision);
        return PCM_OK;
    });
}

double pcm_dynamic_threshold(double e) {
    if (!(e >= 0.0)) return 1.0;  // first SCF step (or NaN): delta = 1
    if (e == 0.0) return 1e-10;
    double d = std::pow(0.1 * e, 1.0 / 1.07);
    return std::min(1.0, std::max(1e-10, d));
}

void pcm_default_threshold_policy(pcm_threshold_policy *p, int kind) {
    if (!p) return;
    p->kind = kind;
    p->delta = 1e-6;
    p->scale = 1e4;
    p->switch_at = 1e-3;
    p->switched = 0;
}

double pcm_cg_threshold(pcm_threshold_policy *p, double e) {
    if (!p) return -1.0;
    switch (p->kind) {
    case PCM_THRESH_FIXED:
        return is_fin(p->delta) && p->delta > 0.0 ? p->delta : -1.0;
    case PCM_THRESH_TWO_DELTA:
        if (!is_fin(p->delta) || !(p->delta > 0.0) || !is_fin(p->scale) || !(p->scale >= 1.0) ||
            !is_fin(p->switch_at) || !(p->switch_at >= 0.0))
            return -1.0;
        // the switch to the tight threshold is made once, when the DIIS error has reached switch_at
        if (!p->switched && e >= 0.0 && e <= p->switch_at) p->switched = 1;
        return p->switched ? p->delta : p->scale * p->delta;
    case PCM_THRESH_DYNAMIC:
        return pcm_dynamic_threshold(e);
    default:
        return -1.0;
    }
}

int pcm_rbj_partition(int M, const double *r, const double *zeta, int l, unsigned long long seed, int *perm,
                      int *blk_off) {
    try {
        return host_rbj_partition(M, r, zeta, l, seed, perm, blk_off);
    } catch (...) {
        return -1;
    }
}

int pcm_octree_partition(int M, const double *r, int leaf_max, int *perm, int *blk_off) {
    try {
        return host_octree_partition(M, r, leaf_max, perm, blk_off);
    } catch (...) {
        return -1;
    }
}

__global__ void k_owner_sph(const int *__restrict__ keep, int M, int nsph, int *__restrict__ owner,
                            int *__restrict__ sph) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    if (owner) owner[k] = keep[k] / nsph;
    if (sph) sph[k] = keep[k] % nsph;
}

pcm_status pcm_surface_get(pcm_ctx *ctx, const pcm_mol *mol, double *r, double *zeta, double *S, double *Akk,
                           int *owner, int *sph) {
    if (!ctx) return PCM_E_ARG;
    if (!mol) return fail(ctx, PCM_E_ARG, "NULL molecule");
    if (any_misaligned(r, zeta, S, Akk)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    if (((uintptr_t)owner | (uintptr_t)sph) & 3) return fail(ctx, PCM_E_ARG, "device int arrays must be 4-byte aligned");
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        const size_t M = mol->M;
        if (r)
            HIP_OK(hipMemcpy2DAsync(r, 3 * sizeof(double), mol->pti64.p, sizeof(PtInt<double>), 3 * sizeof(double), M,
                                    hipMemcpyDeviceToDevice, ctx->stream));
        if (zeta) HIP_OK(hipMemcpyAsync(zeta, mol->zeta.p, M * 8, hipMemcpyDeviceToDevice, ctx->stream));
        if (S) HIP_OK(hipMemcpyAsync(S, mol->S.p, M * 8, hipMemcpyDeviceToDevice, ctx->stream));
        if (Akk) HIP_OK(hipMemcpyAsync(Akk, mol->Akk.p, M * 8, hipMemcpyDeviceToDevice, ctx->stream));
        if (owner || sph) {
            k_owner_sph<<<grid_for(M, 256), 256, 0, ctx->stream>>>(mol->keep.p, (int)M, mol->nsph, owner, sph);
            HIP_LAUNCH_OK();
        }
        return PCM_OK;
    });
}

pcm_status pcm_mol_sizes(const pcm_mol *mol, int *M, int *nbf, int *n_atoms, long long *pairs_fock,
                         long long *pairs_esp, long long *sp_fock, long long *sp_esp) {
    if (!mol) return PCM_E_ARG;
    if (M) *M = mol->M;
    if (nbf) *nbf = mol->nbf;
    if (n_atoms) *n_atoms = mol->N;
    // with a precision split the weak lists are empty unless PCM_DYNAMIC built them
    for (int c = 0; c < NCLS; ++c) {
        if (pairs_fock)
            pairs_fock[c] = mol->fock.cls_off[c + 1] - mol->fock.cls_off[c] + mol->fock_w.cls_off[c + 1] -
                            mol->fock_w.cls_off[c];
        if (pairs_esp)
            pairs_esp[c] =
                mol->esp.cls_off[c + 1] - mol->esp.cls_off[c] + mol->esp_w.cls_off[c + 1] - mol->esp_w.cls_off[c];
        if (sp_fock) sp_fock[c] = mol->fock.sp_union[c];
        if (sp_esp) sp_esp[c] = mol->esp.sp_union[c];
    }
    return PCM_OK;
}

pcm_status pcm_pair_list(pcm_ctx *ctx, const pcm_mol *mol, int which, int *cls, int *a, int *b, int *i, int *j) {
    if (!ctx) return PCM_E_ARG;
    if (!mol || !cls || !a || !b || !i || !j || (which != 0 && which != 1))
        return fail(ctx, PCM_E_ARG, "bad argument");
    const PairList &pl = which == 0 ? mol->fock : mol->esp;
    const PairList &pw = which == 0 ? mol->fock_w : mol->esp_w;  // empty unless PCM_DYNAMIC split it
    return guarded(ctx, [&]() -> pcm_status {
        // entries (shell pair, i*8+j) of both parts, merged back into list order
        auto fetch = [&](const PairList &l) {
            std::vector<std::pair<int, int>> e(l.n);
            std::vector<int> es(l.n), ei(l.n);
            if (l.n) {
                HIP_OK(hipMemcpyAsync(es.data(), l.ent_sp.p, l.n * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
                HIP_OK(hipMemcpyAsync(ei.data(), l.ent_ij.p, l.n * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
                HIP_OK(hipStreamSynchronize(ctx->stream));
            }
            for (long long t = 0; t < l.n; ++t) e[t] = {es[t], ei[t]};
            return e;
        };
        const auto e1 = fetch(pl), e2 = fetch(pw);
        std::vector<std::pair<int, int>> ent;
        ent.reserve(e1.size() + e2.size());
        std::merge(e1.begin(), e1.end(), e2.begin(), e2.end(), std::back_inserter(ent));
        const long long n = (long long)ent.size();
        std::vector<int> es(n), ei(n);
        for (long long t = 0; t < n; ++t) {
            es[t] = ent[t].first;
            ei[t] = ent[t].second;
        }
        for (long long t = 0; t < n; ++t) {
            int sp = es[t];
            int c = 0;
            while (c + 1 < NCLS && sp >= mol->sp_cls_off[c + 1]) ++c;
            cls[t] = c;
            a[t] = mol->h_spa[sp];
            b[t] = mol->h_spb[sp];
            i[t] = ei[t] >> 3;
            j[t] = ei[t] & 7;
        }
        return PCM_OK;
    });
}

pcm_status pcm_profile_enable(pcm_ctx *ctx, int on) {
    if (!ctx) return PCM_E_ARG;
    for (auto &r : ctx->prof_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->prof_recs.clear();
    ctx->prof_agg.clear();
    ctx->prof = on != 0;
    return PCM_OK;
}

int pcm_profile_collect(pcm_ctx *ctx) {
    if (!ctx) return -1;
    if (ctx->stream || ctx->dev_ready) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) return -1;
    }
    for (auto &r : ctx->prof_recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.f;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        bool found = false;
        for (auto &g : ctx->prof_agg)
            if (g.name == r.name) {
                g.ms += ms;
                g.launches += 1;
                g.work += r.work;
                found = true;
                break;
            }
        if (!found) ctx->prof_agg.push_back(ProfAgg{r.name, (double)ms, 1, r.work});
    }
    ctx->prof_recs.clear();
    return (int)ctx->prof_agg.size();
}

pcm_status pcm_profile_entry(const pcm_ctx *ctx, int i, char *name, int name_cap, double *ms, long long *launches,
                             double *work) {
    if (!ctx || i < 0 || i >= (int)ctx->prof_agg.size()) return PCM_E_ARG;
    const ProfAgg &g = ctx->prof_agg[i];
    if (name && name_cap > 0) {
        std::strncpy(name, g.name.c_str(), name_cap - 1);
        name[name_cap - 1] = 0;
    }
    if (ms) *ms = g.ms;
    if (launches) *launches = g.launches;
    if (work) *work = g.work;
    return PCM_OK;
}

void pcm_mol_destroy(pcm_mol *mol) {
    if (!mol) return;
    if (mol->graph) graph_drop(mol->graph);
    release_mol(mol);
    delete mol;
}

pcm_status pcm_batch_create(pcm_ctx *ctx, pcm_mol *const *mols, int n, pcm_batch **out) {
    if (!ctx) return PCM_E_ARG;
    if (!out) return fail(ctx, PCM_E_ARG, "NULL out");
    *out = nullptr;
    if (!mols || n < 1) return fail(ctx, PCM_E_ARG, "a batch needs n >= 1 molecules");
    std::vector<pcm_mol *> v(mols, mols + n);
    for (int i = 0; i < n; ++i) {
        if (!v[i]) return fail(ctx, PCM_E_ARG, "NULL molecule in batch");
        if (v[i]->owner_ctx != ctx) return fail(ctx, PCM_E_ARG, "molecule built on another context");
        if (v[i]->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph (destroy the graph first)");
        for (int j = 0; j < i; ++j)
            if (v[j] == v[i]) return fail(ctx, PCM_E_ARG, "molecule listed twice in batch");
    }
    return guarded(ctx, [&]() -> pcm_status {
        pcm_batch *b = new pcm_batch();
        b->mols = v;
        b->solve = solve_batch_new(v);
        *out = b;
        return PCM_OK;
    });
}

void pcm_batch_destroy(pcm_batch *batch) {
    if (!batch) return;
    if (batch->graph) graph_drop(batch->graph);
    if (batch->solve) solve_batch_free(batch->solve);
    delete batch;
}

pcm_status pcm_esp_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *P, double *const *c,
                           double *const *bz) {
    if (!ctx) return PCM_E_ARG;
    if (!batch || !P || !c) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (batch->graph) return fail(ctx, PCM_E_STATE, "batch is bound to a captured graph (destroy the graph first)");
    const int n = (int)batch->mols.size();
    for (int i = 0; i < n; ++i) {
        if (!P[i] || !c[i]) return fail(ctx, PCM_E_ARG, "NULL matrix or vector in batch");
        if (any_misaligned(P[i], c[i], bz ? bz[i] : nullptr))
            return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    }
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        for (int i = 0; i < n; ++i) density_list(ctx, batch->mols[i], P[i]);
        run_esp_batch(ctx, batch->mols, std::vector<double *>(c, c + n), ctx->prm.precision);
        if (bz)
            for (int i = 0; i < n; ++i)
                if (bz[i]) run_bz(ctx, batch->mols[i], bz[i]);
        return PCM_OK;
    });
}

pcm_status pcm_fock_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *q, double *const *F) {
    if (!ctx) return PCM_E_ARG;
    if (!batch || !q || !F) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (batch->graph) return fail(ctx, PCM_E_STATE, "batch is bound to a captured graph (destroy the graph first)");
    const int n = (int)batch->mols.size();
    for (int i = 0; i < n; ++i) {
        if (!q[i] || !F[i]) return fail(ctx, PCM_E_ARG, "NULL matrix or vector in batch");
        if (any_misaligned(q[i], F[i])) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    }
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        run_fock_batch(ctx, batch->mols, std::vector<const double *>(q, q + n), std::vector<double *>(F, F + n),
                       ctx->prm.precision);
        return PCM_OK;
    });
}

pcm_status pcm_grad_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *P, const double *const *q,
                            double *const *g_nuc, double *const *g_surf) {
    if (!ctx) return PCM_E_ARG;
    if (!batch || !P || !q || !g_nuc || !g_surf) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (batch->graph) return fail(ctx, PCM_E_STATE, "batch is bound to a captured graph (destroy the graph first)");
    const int n = (int)batch->mols.size();
    for (int i = 0; i < n; ++i) {
        if (!P[i] || !q[i] || !g_nuc[i] || !g_surf[i]) return fail(ctx, PCM_E_ARG, "NULL matrix or vector in batch");
        if (any_misaligned(P[i], q[i], g_nuc[i], g_surf[i]))
            return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    }
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        for (int i = 0; i < n; ++i) density_list(ctx, batch->mols[i], P[i]);
        run_grad_batch(ctx, batch->mols, std::vector<const double *>(P, P + n), std::vector<const double *>(q, q + n),
                       std::vector<double *>(g_nuc, g_nuc + n), std::vector<double *>(g_surf, g_surf + n),
                       ctx->prm.precision);
        return PCM_OK;
    });
}

pcm_status pcm_solve_batched(pcm_ctx *ctx, pcm_batch *batch, const double *const *v, const pcm_solve_opts *opts,
                             double *const *q, pcm_solve_info *info) {
    if (!ctx) return PCM_E_ARG;
    if (!batch || !v || !q) return fail(ctx, PCM_E_ARG, "NULL argument");
    if (batch->graph) return fail(ctx, PCM_E_STATE, "batch is bound to a captured graph (destroy the graph first)");
    const int n = (int)batch->mols.size();
    for (int i = 0; i < n; ++i) {
        if (!v[i] || !q[i]) return fail(ctx, PCM_E_ARG, "NULL vector in batch");
        if (any_misaligned(v[i], q[i])) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    }
    pcm_solve_opts o;
    pcm_status vs = check_solve_opts(ctx, opts, o);
    if (vs != PCM_OK) return vs;
    return guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        std::vector<const double *> vv(v, v + n);
        std::vector<double *> qq(q, q + n);
        pcm_status st = solve_batch_run(ctx, *batch->solve, vv, qq, o, info);
        if (st == PCM_E_NOCONV) ctx->err = "max_iter reached before the residual threshold";
        return st;
    });
}

}  // extern "C"
