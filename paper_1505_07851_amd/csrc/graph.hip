// One solvation pass of a whole batch as a single hipGraph (the batching form of the hot path):
// for every molecule, the density coefficients of the Eq. 18 list rebuilt from the current P,
// c = L P (Eqs. 5-6) and Bz (Eq. 4), the preconditioned CG solve of Eq. 1 (Sec. 4b) with a fixed
// iteration budget, the Eq. 13 energy and F += L^T q (Eq. 10).  Capture does every host step
// first -- screening, chunk choice, descriptor and solver tables, the block-Jacobi partition and
// inverses, the matvec grid -- and records the launches; a replay is one hipGraphLaunch.
//
// The graph holds the molecules' list, record and workspace buffers by address, so the
// molecules and the batch refuse every other call until the graph is destroyed.
#include "pcm_internal.h"

#include <memory>
#include <mutex>
#include <set>

struct pcm_graph {
    pcm_ctx *ctx = nullptr;
    pcm_batch *batch = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    std::vector<std::unique_ptr<DevBuf<unsigned char>>> bufs;  // descriptor tables of the passes
    GraphSolveBufs *sb = nullptr;
    double tol = 0.0;
    int budget = 0;
    size_t nodes = 0;
};

// live graphs: destroying a batch or a molecule drops its graph, and a later destroy, launch or
// info call on that handle is then refused instead of touching freed memory
static std::mutex g_live_mu;
static std::set<pcm_graph *> g_live;

static bool live(pcm_graph *g) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(g) != 0;
}

static void graph_release(pcm_graph *g) {
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.erase(g);
    }
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    for (auto &b : g->bufs) b->release();
    if (g->sb) graph_solve_bufs_free(g->sb);
    if (g->batch) {
        for (pcm_mol *m : g->batch->mols)
            if (m->graph == g) m->graph = nullptr;
        if (g->batch->graph == g) g->batch->graph = nullptr;
    }
    delete g;
}

void graph_drop(pcm_graph *g) {
    if (!g || !live(g)) return;
    if (g->ctx && g->ctx->stream) (void)hipStreamSynchronize(g->ctx->stream);
    graph_release(g);
}

static bool misaligned8(const void *p) { return ((uintptr_t)p & 7) != 0; }

extern "C" {

pcm_status pcm_graph_capture(pcm_ctx *ctx, pcm_batch *batch, const double *const *P, double *const *c,
                             double *const *bz, double *const *q, double *const *F, double *E,
                             const pcm_solve_opts *opts, pcm_graph **out) {
    if (!ctx) return PCM_E_ARG;
    if (!batch || !P || !c || !bz || !q || !F || !E || !out) return fail(ctx, PCM_E_ARG, "NULL argument");
    *out = nullptr;
    const int n = (int)batch->mols.size();
    if (misaligned8(E)) return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    for (int i = 0; i < n; ++i) {
        if (!P[i] || !c[i] || !bz[i] || !q[i] || !F[i]) return fail(ctx, PCM_E_ARG, "NULL matrix or vector in batch");
        if (misaligned8(P[i]) || misaligned8(c[i]) || misaligned8(bz[i]) || misaligned8(q[i]) || misaligned8(F[i]))
            return fail(ctx, PCM_E_ARG, "device arrays must be 8-byte aligned");
    }
    pcm_solve_opts o;
    pcm_status vs = check_solve_opts(ctx, opts, o);
    if (vs != PCM_OK) return vs;
    if (o.precision != PCM_FP64)
        return fail(ctx, PCM_E_UNSUPPORTED, "the captured solve is FP64 PCG (mixed refinement needs host decisions)");
    if (o.max_iter > 100000) return fail(ctx, PCM_E_ARG, "iteration budget above 100000");
    if (batch->graph) return fail(ctx, PCM_E_STATE, "batch is already bound to a captured graph");
    for (pcm_mol *m : batch->mols)
        if (m->graph) return fail(ctx, PCM_E_STATE, "molecule is bound to a captured graph");
    pcm_graph *g = new (std::nothrow) pcm_graph();
    if (!g) return fail(ctx, PCM_E_ALLOC, "host allocation failed");
    g->ctx = ctx;
    g->tol = o.tol;
    g->budget = o.max_iter;
    pcm_status st = guarded(ctx, [&]() -> pcm_status {
        ctx_ensure_device(ctx);
        const int prec = ctx->prm.precision;
        std::vector<pcm_mol *> mols = batch->mols;
        Launches L;
        // density lists screened with the P of the capture; each replay rebuilds their records
        for (int i = 0; i < n; ++i) {
            density_list(ctx, mols[i], P[i]);
            if (prec == PCM_DYNAMIC) {
                density_record_launches(ctx, mols[i], mols[i]->esp, P[i], PCM_FP64, L);
                density_record_launches(ctx, mols[i], mols[i]->esp_w, P[i], PCM_MIXED, L);
            } else {
                density_record_launches(ctx, mols[i], mols[i]->esp, P[i], PCM_FP64, L);
            }
        }
        esp_batch_launches(ctx, mols, std::vector<double *>(c, c + n), prec, g->bufs, L);
        for (int i = 0; i < n; ++i) bz_launches(ctx, mols[i], bz[i], L);
        g->sb = graph_solve_bufs_new();
        solve_graph_launches(ctx, *batch->solve, std::vector<const double *>(bz, bz + n),
                             std::vector<const double *>(c, c + n), std::vector<double *>(q, q + n), E, o,
                             o.max_iter, *g->sb, L);
        fock_batch_launches(ctx, mols, std::vector<const double *>(q, q + n), std::vector<double *>(F, F + n), prec,
                            g->bufs, L);
        HIP_OK(hipStreamSynchronize(ctx->stream));  // every table upload of the set-up has landed
        HIP_OK(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIP_OK(hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed));
        try {
            L.run(ctx, g->cap, false);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(g->cap, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        HIP_OK(hipStreamEndCapture(g->cap, &graph));
        size_t nn = 0;
        (void)hipGraphGetNodes(graph, nullptr, &nn);
        g->nodes = nn;
        hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_OK(e);
        return PCM_OK;
    });
    if (st != PCM_OK) {
        graph_release(g);
        return st;
    }
    g->batch = batch;
    batch->graph = g;
    for (pcm_mol *m : batch->mols) m->graph = g;
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(g);
    }
    *out = g;
    return PCM_OK;
}


pcm_status pcm_graph_launch(pcm_ctx *ctx, pcm_graph *g) {
    if (!ctx) return PCM_E_ARG;
    if (!g || !live(g) || g->ctx != ctx) return fail(ctx, PCM_E_ARG, "graph NULL, destroyed or of another context");
    return guarded(ctx, [&]() -> pcm_status {
        HIP_OK(hipGraphLaunch(g->exec, ctx->stream));
        return PCM_OK;
    });
}

pcm_status pcm_graph_info(pcm_ctx *ctx, pcm_graph *g, pcm_solve_info *info, long long *nodes) {
    if (!ctx) return PCM_E_ARG;
    if (!g || !live(g) || g->ctx != ctx) return fail(ctx, PCM_E_ARG, "graph NULL, destroyed or of another context");
    if (nodes) *nodes = (long long)g->nodes;
    return guarded(ctx, [&]() -> pcm_status {
        const int n = (int)g->batch->mols.size();
        std::vector<int> conv(n, 0);
        solve_graph_info(ctx, *g->batch->solve, g->tol, info, conv.data());
        for (int i = 0; i < n; ++i)
            if (!conv[i]) {
                ctx->err = "a molecule did not reach the residual threshold within the iteration budget";
                return PCM_E_NOCONV;
            }
        return PCM_OK;
    });
}

void pcm_graph_destroy(pcm_graph *g) { graph_drop(g); }

}  // extern "C"
