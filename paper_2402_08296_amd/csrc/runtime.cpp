// Host runtime of the DDM-GNN solver: contexts, models, problems, batches of
// problems solved in lockstep, the solve driver (graph-captured chunks of
// iterations, host polls of the per-problem converged flags) and the C ABI
// declared in include/ddmgnn.h (the serving entry points are in server.cpp).
#include "runtime.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace ddmgnn {

namespace {
thread_local std::string g_err;
std::atomic<uint64_t> g_next_id{1};
}  // namespace

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// ------------------------------------------------------------------ batch
struct Batch {
    ddmgnn_ctx* ctx = nullptr;
    std::vector<ddmgnn_problem*> probs;
    std::vector<uint64_t> ids;
    std::shared_ptr<ModelDev> model;
    std::vector<DevProb> views;        // host copy of tab
    DevBuf<DevProb> tab;               // table of the solve
    DevBuf<DevProb> hook;              // one-problem table of the entry points that redirect vectors
    // DSS work lists, (problem, sub-mesh) by decreasing sub-mesh size:
    // all sub-meshes; those of problems that fit the MFMA kernel; the others.
    // (the VALU lists hold sub-meshes of at most kMaxSubNodes nodes; work_big the larger ones,
    // which run the global-memory form of the VALU kernel in every precision)
    DevBuf<int2> work_all, work_mfma, work_rest, work_valu, work_big;
    int n_all = 0, n_mfma = 0, n_rest = 0, n_valu = 0, n_big = 0;
    // the MFMA list split by workgroup size: sub-meshes that run two per compute
    // unit in MFMA_SMALL_BLOCK-thread workgroups, and the rest; dynamic LDS of each launch
    DevBuf<int2> work_mfma_small;
    int n_mfma_small = 0;
    size_t lds_mfma = 0, lds_mfma_small = 0;
    int max_k_all = 0, max_k_rest = 0, max_k_valu = 0;
    DevBuf<int2> vec_blk;              // (problem, local workgroup)
    int n_vec = 0;
    DevBuf<int2> coarse_rows;          // (problem, row)
    int n_coarse = 0;
    DevBuf<int2> sub_blk;              // subset of vec_blk (init and residual of some problems)
    int n_sub_blk = 0;
    DevBuf<int> sub_list;              // the problems of that subset (their finalize workgroups)
    int n_sub_list = 0;
    DevBuf<KState> st_gather;
    KState* host_st = nullptr;         // pinned, one per problem
    hipGraphExec_t graph = nullptr;    // captured chunk of iterations
    uint64_t graph_key = 0;
    ~Batch() {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (host_st) (void)hipHostFree(host_st);
    }
};

namespace {

DevProb make_view(ddmgnn_problem* P) {
    DevProb v{};
    v.rowptr = P->rowptr.p; v.col = P->col.p; v.val = P->val.p; v.b = P->b.p; v.u0 = P->u0.p;
    v.dirichlet = P->dirichlet.p;
    v.sub_ptr = P->sub_ptr.p; v.sub_nodes = P->sub_nodes.p; v.weights = P->weights.p;
    v.edge_ptr = P->edge_ptr.p; v.edge_src = P->edge_src.p; v.edge_nd = P->edge_nd.p; v.erec = P->erec.p;
    v.epad_sub = P->epad_sub.p;
    v.tiles = P->tiles.p; v.xy64 = P->xy64.p; v.xyc32 = P->xyc32.p;
    v.node_ptr = P->node_ptr.p; v.node_slots = P->node_slots.p; v.slot_sub = P->slot_sub.p; v.a0inv = P->a0inv.p;
    v.lu_inv = P->lu_inv.p; v.lu_off = P->lu_off.p;
    v.gm_v = P->gm_v.p; v.gm_z = P->gm_z.p; v.gm_part = P->gm_part.p; v.gm_small = P->gm_small.p;
    v.u = P->u.p; v.r = P->r.p; v.z = P->z.p; v.c_in = nullptr;
    const int64_t n = P->hs.n;
    for (int i = 0; i <= MAX_M; ++i) {
        v.p[i] = P->ring.p + (size_t)i * n;
        v.q[i] = P->ring.p + (size_t)(MAX_M + 1 + i) * n;
    }
    v.s = P->s.p; v.y0 = P->y0.p; v.y = P->y.p; v.local = P->local.p;
    v.qg64 = P->qglobal64.p; v.hg64 = P->hglobal64.p; v.qg32 = P->qglobal32.p;
    v.hg32 = P->hglobal32.p; v.c64 = P->cglobal.p; v.c32 = reinterpret_cast<float*>(P->cglobal.p);
    v.st = P->st.p;
    v.partials = P->partials.p;
    v.rtol = P->rtol;
    v.max_it = P->max_it;
    v.n = (int)n;
    v.K = P->hs.K;
    v.nblk = problem_vec_blocks(P);
    return v;
}

hipError_t upload_async(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

template <typename T>
int upload_list(DevBuf<T>& buf, const std::vector<T>& v, hipStream_t s) {
    if (buf.n < v.size() || !buf.p) HIP_TRY(buf.alloc(std::max<size_t>(v.size(), 1)));
    HIP_TRY(upload_async(buf.p, v.data(), v.size() * sizeof(T), s));
    return DDMGNN_OK;
}

bool valu_q_in_lds(int max_k, int precision, int d) {
    const size_t esz = precision == DDMGNN_FP64 ? sizeof(double) : sizeof(float);
    return (size_t)max_k * 2 * d * esz + 1024 <= LDS_LIMIT;
}

size_t valu_shmem(int max_k, int precision, int d) {
    const size_t esz = precision == DDMGNN_FP64 ? sizeof(double) : sizeof(float);
    return (size_t)max_k * 2 * d * esz;
}

// Exact local solves: the inverses of R_i A R_i^T, assembled from the problem's
// device matrix and inverted on the device (one workgroup per sub-mesh).
// In-place inverses of a batch of SPD matrices on the device (orders k, matrix
// m at base + off_dev[m]); E_NOT_SPD when a pivot fails.
int gj_invert_batch(const std::vector<int32_t>& k, double* base, const int64_t* off_dev, const double* diag0,
                    hipStream_t s, GjBufs& g) {
    const GjPlan plan(k);
    HIP_TRY(g.order.upload(plan.order.data(), plan.order.size(), s));
    HIP_TRY(g.cprefix.upload(plan.cprefix.data(), plan.cprefix.size(), s));
    HIP_TRY(g.tprefix.upload(plan.tprefix.data(), plan.tprefix.size(), s));
    HIP_TRY(g.prow.upload(plan.prow.data(), plan.prow.size(), s));
    HIP_TRY(g.scratch.alloc(plan.scratch_doubles()));
    HIP_TRY(g.status.alloc(1));
    HIP_TRY(hipMemsetAsync(g.status.p, 0, sizeof(int), s));
    const GjPlanDev dev{g.order.p, g.cprefix.p, g.tprefix.p, g.prow.p};
    HIP_TRY(launch_gj_invert(plan, dev, base, off_dev, g.scratch.p, diag0, g.status.p, s));
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, g.status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return bad ? DDMGNN_E_NOT_SPD : DDMGNN_OK;
}

int prepare_lu(ddmgnn_problem* P) {
    HIP_TRY(prepare_lu_local());
    if (P->lu_inv.p) return DDMGNN_OK;
    hipStream_t s = P->ctx->stream;
    const auto& hs = P->hs;
    std::vector<int64_t> off((size_t)hs.K + 1, 0);
    for (int32_t i = 0; i < hs.K; ++i) {
        const int64_t k = hs.sub_ptr[i + 1] - hs.sub_ptr[i];
        off[i + 1] = off[i] + k * lu_ld(k);
    }
    auto build = [&]() -> int {
        DevBuf<int64_t> sub_ptr64;
        HIP_TRY(sub_ptr64.upload(hs.sub_ptr.data(), hs.sub_ptr.size(), s));
        HIP_TRY(P->lu_off.upload(off.data(), off.size(), s));
        HIP_TRY(P->lu_inv.alloc((size_t)std::max<int64_t>(off[hs.K], 1)));
        HIP_TRY(launch_lu_assemble(P->rowptr.p, P->col.p, P->val.p, sub_ptr64.p, P->sub_nodes.p, P->lu_off.p,
                                   P->lu_inv.p, hs.K, s));
        std::vector<int32_t> k((size_t)hs.K);
        for (int32_t i = 0; i < hs.K; ++i) k[i] = (int32_t)(hs.sub_ptr[i + 1] - hs.sub_ptr[i]);
        GjBufs g;
        const int rc = gj_invert_batch(k, P->lu_inv.p, P->lu_off.p, nullptr, s, g);
        if (rc == DDMGNN_E_NOT_SPD) return fail(rc, "a local matrix R_i A R_i^T is not positive definite");
        return rc;
    };
    if (int rc = build()) {  // leave no half-built inverses behind
        P->lu_inv.reset();
        P->lu_off.reset();
        return rc;
    }
    P->device_bytes += (size_t)off[hs.K] * sizeof(double) + off.size() * sizeof(int64_t);
    return DDMGNN_OK;
}

// Training structures of a problem: per slot, its row of A_i = R_i A R_i^T
// (local columns, ascending) and the in-edges it sends (ordered by edge index).
int prepare_train(ddmgnn_problem* P) {
    if (P->lm_ptr.p) return DDMGNN_OK;
    hipStream_t s = P->ctx->stream;
    const auto& hs = P->hs;
    std::vector<int32_t> rowptr(hs.n + 1), col(hs.nnz), sub_nodes(hs.sk);
    std::vector<double> val(hs.nnz);
    HIP_TRY(hipMemcpyAsync(rowptr.data(), P->rowptr.p, rowptr.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(col.data(), P->col.p, col.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(val.data(), P->val.p, val.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sub_nodes.data(), P->sub_nodes.p, sub_nodes.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> lm_ptr(hs.sk + 1, 0), oe_ptr(hs.sk + 1, 0), oe_edge(std::max<int64_t>(hs.n_edges, 1));
    std::vector<uint16_t> lm_col, oe_recv(std::max<int64_t>(hs.n_edges, 1));
    std::vector<float> lm_val;
    lm_col.reserve((size_t)hs.sk * 7);
    lm_val.reserve((size_t)hs.sk * 7);
    for (int32_t i = 0; i < hs.K; ++i) {
        const int64_t b = hs.sub_ptr[i], e = hs.sub_ptr[i + 1];
        const int32_t* first = sub_nodes.data() + b;
        const int32_t* last = sub_nodes.data() + e;
        for (int64_t q = b; q < e; ++q) {
            const int32_t j = sub_nodes[q];
            for (int32_t a = rowptr[j]; a < rowptr[j + 1]; ++a) {
                const int32_t* f = std::lower_bound(first, last, col[a]);
                if (f == last || *f != col[a]) continue;
                lm_col.push_back((uint16_t)(f - first));
                lm_val.push_back((float)val[a]);
            }
            lm_ptr[q + 1] = (int32_t)lm_col.size();
        }
        for (int64_t q = b; q < e; ++q)
            for (int64_t t = hs.edge_ptr[q]; t < hs.edge_ptr[q + 1]; ++t) oe_ptr[b + hs.edge_src[t] + 1]++;
    }
    if (lm_col.size() >= (size_t)INT32_MAX) return fail(DDMGNN_E_INVALID, "local matrices too large");
    for (int64_t q = 0; q < hs.sk; ++q) oe_ptr[q + 1] += oe_ptr[q];
    std::vector<int32_t> fill(oe_ptr.begin(), oe_ptr.end() - 1);
    for (int32_t i = 0; i < hs.K; ++i) {
        const int64_t b = hs.sub_ptr[i], e = hs.sub_ptr[i + 1];
        for (int64_t q = b; q < e; ++q)
            for (int64_t t = hs.edge_ptr[q]; t < hs.edge_ptr[q + 1]; ++t) {
                const int32_t at = fill[b + hs.edge_src[t]]++;
                oe_edge[at] = (int32_t)t;
                oe_recv[at] = (uint16_t)(q - b);
            }
    }
    HIP_TRY(P->lm_ptr.upload(lm_ptr.data(), lm_ptr.size(), s));
    HIP_TRY(P->lm_col.upload(lm_col.data(), std::max<size_t>(lm_col.size(), 1), s));
    HIP_TRY(P->lm_val.upload(lm_val.data(), std::max<size_t>(lm_val.size(), 1), s));
    HIP_TRY(P->oe_ptr.upload(oe_ptr.data(), oe_ptr.size(), s));
    HIP_TRY(P->oe_edge.upload(oe_edge.data(), oe_edge.size(), s));
    HIP_TRY(P->oe_recv.upload(oe_recv.data(), oe_recv.size(), s));
    P->device_bytes += lm_ptr.size() * 4 + lm_col.size() * 2 + lm_val.size() * 4 + oe_ptr.size() * 4 +
                       oe_edge.size() * 6;
    return DDMGNN_OK;
}

// Whether the BF16 MFMA kernel runs sub-mesh `sub` of P (the model has the
// paper's latent width and the sub-mesh fits the kernel's node and LDS budgets).
bool mfma_runs_sub(const ddmgnn_problem* P, int sub) {
    return P->model->mfma && P->mfma_need[(size_t)sub] <= MFMA_LDS_LIMIT;
}
// Whether every sub-mesh of P runs on the VALU kernels under BF16.
bool all_valu_bf16(const ddmgnn_problem* P) {
    for (int i = 0; i < P->hs.K; ++i)
        if (mfma_runs_sub(P, i)) return false;
    return true;
}
bool any_valu_bf16(const ddmgnn_problem* P) {
    for (int i = 0; i < P->hs.K; ++i)
        if (!mfma_runs_sub(P, i)) return true;
    return false;
}

int prepare_fgmres(Batch& B, int R, bool& changed) {
    for (ddmgnn_problem* P : B.probs) {
        if (P->gm_R >= R) continue;
        const size_t n = (size_t)P->hs.n;
        P->device_bytes -= P->gm_R ? fgmres_bytes(P->hs.n, P->gm_R) : 0;
        P->gm_R = 0;
        HIP_TRY(P->gm_v.alloc((size_t)(R + 1) * n));
        HIP_TRY(P->gm_z.alloc((size_t)R * n));
        HIP_TRY(P->gm_part.alloc((size_t)(R + 1) * VEC_GRID));
        HIP_TRY(P->gm_small.alloc((size_t)R * R + 6 * R + 2));
        P->gm_R = R;
        P->device_bytes += fgmres_bytes(P->hs.n, R);
        changed = true;
    }
    return DDMGNN_OK;
}

// Allocates what the DSS launches of this precision need (fallback storage,
// LDS attributes). Not allowed during stream capture; returns true in
// `changed` when a problem's buffers moved (the table must be re-uploaded).
int prepare_dss(Batch& B, int precision, bool& changed) {
    changed = false;
    const bool bf16 = precision == DDMGNN_BF16;
    if (bf16 && B.n_mfma + B.n_mfma_small) HIP_TRY(prepare_dss_mfma(MFMA_LDS_LIMIT));
    const int valu_prec = bf16 ? DDMGNN_FP32 : precision;
    const bool f64 = valu_prec == DDMGNN_FP64;
    const int d = B.model->d;
    // sub-meshes beyond kMaxSubNodes: h, c and Q per slot in global memory
    for (ddmgnn_problem* P : B.probs) {
        if (!P->has_big) continue;
        const size_t sk = (size_t)P->hs.sk;
        if (f64 && P->qglobal64.n < sk * 2 * d) {
            HIP_TRY(P->qglobal64.alloc(sk * 2 * d));
            changed = true;
        }
        if (!f64 && P->qglobal32.n < sk * 2 * d) {
            HIP_TRY(P->qglobal32.alloc(sk * 2 * d));
            changed = true;
        }
        if (f64 && P->hglobal64.n < sk * d) {
            HIP_TRY(P->hglobal64.alloc(sk * d));
            changed = true;
        }
        if (!f64 && P->hglobal32.n < sk * d) {
            HIP_TRY(P->hglobal32.alloc(sk * d));
            changed = true;
        }
        if (P->cglobal.n < sk) {
            HIP_TRY(P->cglobal.alloc(sk));
            changed = true;
        }
    }
    const int max_k = bf16 ? B.max_k_rest : B.max_k_valu;
    const int n_valu = bf16 ? B.n_rest : B.n_valu;
    if (n_valu == 0) return DDMGNN_OK;
    const bool in_lds = valu_q_in_lds(max_k, valu_prec, d);
    for (ddmgnn_problem* P : B.probs) {
        if (bf16 && !any_valu_bf16(P)) continue;
        const size_t sk = (size_t)P->hs.sk;
        if (!in_lds) {
            if (f64 && P->qglobal64.n < sk * 2 * d) {
                HIP_TRY(P->qglobal64.alloc(sk * 2 * d));
                changed = true;
            }
            if (!f64 && P->qglobal32.n < sk * 2 * d) {
                HIP_TRY(P->qglobal32.alloc(sk * 2 * d));
                changed = true;
            }
        }
        if (f64 && P->hglobal64.n < sk * d) {
            HIP_TRY(P->hglobal64.alloc(sk * d));
            changed = true;
        }
    }
    if (in_lds) HIP_TRY(prepare_dss_valu(valu_prec, d, LDS_LIMIT - 1024));
    return DDMGNN_OK;
}

// Local solves over every sub-mesh of the table: the DSS forward (apply:
// restriction and s r~), or the exact solves of DDM-LU.
int enqueue_dss(Batch& B, const DevProb* tab, int precision, int apply, bool capturing, int local = DDMGNN_LOCAL_GNN) {
    hipStream_t s = B.ctx->launch;
    const ModelDev& M = *B.model;
    const bool check = !capturing;
    if (local == DDMGNN_LOCAL_LU) {
        HIP_TRY(launch_lu_local(tab, B.work_all.p, B.n_all, B.max_k_all, s, check));
        return DDMGNN_OK;
    }
    HIP_TRY(launch_dss_big(tab, B.work_big.p, B.n_big, precision == DDMGNN_BF16 ? DDMGNN_FP32 : precision, M.d,
                           M.kbar, M.alpha, apply, M.theta32.p, M.theta64.p, s, check));
    if (precision == DDMGNN_BF16) {
        DssMfmaArgs a{tab, B.work_mfma.p, M.steps.p, M.dec.p, M.kbar, (float)M.alpha, apply};
        if (B.n_mfma > 0 && B.n_mfma_small > 0) {
            // the two workgroup sizes on two streams, so that either launch's last
            // round overlaps the other's work; joined back before the next kernel
            ddmgnn_ctx* ctx = B.ctx;
            HIP_TRY(hipEventRecord(ctx->fork_ev, s));
            HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
            DssMfmaArgs small = a;
            small.work = B.work_mfma_small.p;
            HIP_TRY(launch_dss_mfma(small, B.n_mfma_small, B.lds_mfma_small, MFMA_SMALL_BLOCK, ctx->side, check));
            HIP_TRY(hipEventRecord(ctx->join_ev, ctx->side));
            HIP_TRY(launch_dss_mfma(a, B.n_mfma, B.lds_mfma, MFMA_BLOCK, s, check));
            HIP_TRY(hipStreamWaitEvent(s, ctx->join_ev, 0));
        } else {
            HIP_TRY(launch_dss_mfma(a, B.n_mfma, B.lds_mfma, MFMA_BLOCK, s, check));
            a.work = B.work_mfma_small.p;
            HIP_TRY(launch_dss_mfma(a, B.n_mfma_small, B.lds_mfma_small, MFMA_SMALL_BLOCK, s, check));
        }
        const bool qlds = valu_q_in_lds(B.max_k_rest, DDMGNN_FP32, M.d);
        HIP_TRY(launch_dss_valu(tab, B.work_rest.p, B.n_rest, DDMGNN_FP32, M.d, qlds, M.kbar, M.alpha, apply,
                                M.theta32.p, M.theta64.p, qlds ? valu_shmem(B.max_k_rest, DDMGNN_FP32, M.d) : 0, s,
                                check));
    } else {
        const bool qlds = valu_q_in_lds(B.max_k_valu, precision, M.d);
        HIP_TRY(launch_dss_valu(tab, B.work_valu.p, B.n_valu, precision, M.d, qlds, M.kbar, M.alpha, apply,
                                M.theta32.p, M.theta64.p, qlds ? valu_shmem(B.max_k_valu, precision, M.d) : 0, s,
                                check));
    }
    return DDMGNN_OK;
}

IterArgs iter_args(const ddmgnn_solve_opts& o, int mode) {
    IterArgs ia{};
    ia.mode = mode;
    ia.m = mode == DDMGNN_FCG ? o.m_max : mode == DDMGNN_FGMRES ? o.restart : 1;
    ia.unweighted = o.prolong == DDMGNN_PROLONG_UNWEIGHTED;
    ia.coarse = o.coarse;
    return ia;
}

// One preconditioner apply z = M(r) over the table (mode < 0: no Krylov dots).
// ev (optional): events recorded after the DSS (ev[1]), coarse (ev[2]) and prolong (ev[3]) launches.
int enqueue_apply(Batch& B, const DevProb* tab, const ddmgnn_solve_opts& o, int mode, hipEvent_t* ev,
                  bool capturing) {
    if (int rc = enqueue_dss(B, tab, o.precision, 1, capturing, o.local_solver)) return rc;
    hipStream_t s = B.ctx->launch;
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    if (o.coarse) HIP_TRY(launch_coarse(tab, B.coarse_rows.p, B.n_coarse, s, !capturing));
    if (ev) HIP_TRY(hipEventRecord(ev[2], s));
    HIP_TRY(launch_prolong(tab, B.vec_blk.p, B.n_vec, (int)B.probs.size(), iter_args(o, mode), s, !capturing));
    if (ev) HIP_TRY(hipEventRecord(ev[3], s));
    return DDMGNN_OK;
}

// One FCG/PCG/CG iteration of every problem of the batch. ev: optional 5
// profiling events (before DSS, after DSS / coarse / prolong, end).
int enqueue_iteration(Batch& B, const ddmgnn_solve_opts& o, hipEvent_t* ev, bool capturing) {
    hipStream_t s = B.ctx->launch;
    const int mode = o.krylov;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    if (mode == DDMGNN_FGMRES) {
        HIP_TRY(launch_fgmres_next(B.tab.p, B.vec_blk.p, B.n_vec, iter_args(o, mode), s, !capturing));
        if (int rc = enqueue_apply(B, B.tab.p, o, mode, ev, capturing)) return rc;
        HIP_TRY(launch_fgmres_step(B.tab.p, B.vec_blk.p, B.n_vec, (int)B.probs.size(), iter_args(o, mode), s,
                                   !capturing));
        if (ev) HIP_TRY(hipEventRecord(ev[4], s));
        return DDMGNN_OK;
    }
    if (mode == DDMGNN_CG) {
        if (ev)
            for (int q = 1; q < 4; ++q) HIP_TRY(hipEventRecord(ev[q], s));
    } else {
        if (int rc = enqueue_apply(B, B.tab.p, o, mode, ev, capturing)) return rc;
    }
    HIP_TRY(launch_krylov(B.tab.p, B.vec_blk.p, B.n_vec, (int)B.probs.size(), iter_args(o, mode), s, !capturing));
    if (ev) HIP_TRY(hipEventRecord(ev[4], s));
    return DDMGNN_OK;
}

uint64_t graph_key(const ddmgnn_solve_opts& o, int count) {
    const int m = o.krylov == DDMGNN_FGMRES ? o.restart : o.m_max;
    return ((uint64_t)o.local_solver << 56) | ((uint64_t)o.krylov << 52) | ((uint64_t)(m & 0xff) << 44) |
           ((uint64_t)o.precision << 40) | ((uint64_t)o.prolong << 38) | ((uint64_t)(o.coarse != 0) << 36) |
           (uint64_t)(uint32_t)count;
}

// Captures `count` iterations of the batch into B.graph (on the context's own
// stream: the caller's stream may be the null stream, which cannot be captured).
int capture_chunk(Batch& B, const ddmgnn_solve_opts& o, int count) {
    ddmgnn_ctx* ctx = B.ctx;
    if (B.graph) {
        (void)hipGraphExecDestroy(B.graph);
        B.graph = nullptr;
        B.graph_key = 0;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed));
    ctx->launch = ctx->cap;
    int crc = 0;
    for (int c = 0; c < count && crc == 0; ++c) crc = enqueue_iteration(B, o, nullptr, true);
    ctx->launch = ctx->stream;
    hipError_t ce = hipStreamEndCapture(ctx->cap, &g);
    if (crc || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(ctx->cap, &cst) == hipSuccess && cst != hipStreamCaptureStatusNone) {
            hipGraph_t g2 = nullptr;
            (void)hipStreamEndCapture(ctx->cap, &g2);
            if (g2) (void)hipGraphDestroy(g2);
        }
        if (crc) return crc;
        HIP_TRY(ce);
    }
    HIP_TRY(hipGetLastError());
    hipError_t ie = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(ie);
    B.graph_key = graph_key(o, count);
    return DDMGNN_OK;
}

int upload_table(Batch& B) {
    B.views.resize(B.probs.size());
    for (size_t i = 0; i < B.probs.size(); ++i) B.views[i] = make_view(B.probs[i]);
    return upload_list(B.tab, B.views, B.ctx->stream);
}

// Workgroup list and problem list of the problems flagged in `which`.
int upload_subset(Batch& B, const std::vector<uint8_t>* which) {
    std::vector<int2> sub;
    std::vector<int> list;
    for (size_t i = 0; i < B.probs.size(); ++i) {
        if (which && !(*which)[i]) continue;
        list.push_back((int)i);
        const int nb = problem_vec_blocks(B.probs[i]);
        for (int b = 0; b < nb; ++b) sub.push_back(make_int2((int)i, b));
    }
    B.n_sub_blk = (int)sub.size();
    B.n_sub_list = (int)list.size();
    if (int rc = upload_list(B.sub_list, list, B.ctx->stream)) return rc;
    return upload_list(B.sub_blk, sub, B.ctx->stream);
}

int solo_batch(ddmgnn_problem* P) {
    if (P->solo) return DDMGNN_OK;
    ddmgnn_problem* one[1] = {P};
    return build_batch(P->ctx, one, 1, P->solo);
}

// Solve every problem of the batch from its u0 with options o.
int solve_batch(ddmgnn_ctx* ctx, Batch& B, const ddmgnn_solve_opts& o, double* const* u_out, ddmgnn_stats* stats) {
    hipStream_t s = ctx->stream;
    const int nb = (int)B.probs.size();
    for (ddmgnn_problem* P : B.probs) {
        P->rtol = o.rtol;
        P->max_it = o.max_it;
    }
    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    struct EvGuard {
        hipEvent_t a, b;
        std::vector<hipEvent_t> v;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            for (auto e : v) (void)hipEventDestroy(e);
        }
    } guard{ev0, ev1, {}};
    if (int rc = batch_begin(B, o, nullptr)) return rc;
    HIP_TRY(hipEventRecord(ev0, s));
    HIP_TRY(launch_init(B.tab.p, B.vec_blk.p, B.n_vec, nullptr, nb, s));
    // Iterations between host polls of the converged flags; a captured chunk
    // is replayed as a whole (problems that finish inside it idle).
    const int check = std::max(1, o.check_every);
    const bool use_graph = o.graph && !o.profile;
    if (o.profile) {
        guard.v.resize((size_t)check * 5);
        for (auto& e : guard.v) HIP_TRY(hipEventCreate(&e));
    }
    double t_dss = 0, t_coarse = 0, t_prolong = 0, t_krylov = 0;
    int n_dss = 0, it = 0, it_seen = 0;
    bool done = o.max_it <= 0;
    while (!done) {
        const int n_chunk = use_graph ? check : std::min(check, o.max_it - it);
        if (use_graph) {
            if (!B.graph || B.graph_key != graph_key(o, n_chunk))
                if (int rc = capture_chunk(B, o, n_chunk)) return rc;
            HIP_TRY(hipGraphLaunch(B.graph, s));
        } else {
            for (int c = 0; c < n_chunk; ++c)
                if (int rc = enqueue_iteration(B, o, o.profile ? &guard.v[(size_t)c * 5] : nullptr, false)) return rc;
        }
        if (int rc = batch_poll(B)) return rc;
        it += n_chunk;
        bool all = true;
        int max_it_done = 0;
        for (int i = 0; i < nb; ++i) {
            all = all && B.host_st[i].done;
            max_it_done = std::max(max_it_done, B.host_st[i].it);
        }
        done = all || it >= o.max_it;
        if (o.profile) {
            // iterations it_seen .. max_it_done-1 did work; later ones exited at once
            const int worked = std::min(n_chunk, std::max(0, max_it_done - it_seen));
            for (int c = 0; c < worked; ++c) {
                hipEvent_t* ev = &guard.v[(size_t)c * 5];
                float a = 0, b = 0, cc = 0, d = 0;
                HIP_TRY(hipEventElapsedTime(&a, ev[0], ev[1]));
                HIP_TRY(hipEventElapsedTime(&b, ev[1], ev[2]));
                HIP_TRY(hipEventElapsedTime(&cc, ev[2], ev[3]));
                HIP_TRY(hipEventElapsedTime(&d, ev[3], ev[4]));
                t_dss += a;
                t_coarse += b;
                t_prolong += cc;
                t_krylov += d;
                if (o.krylov != DDMGNN_CG) ++n_dss;
            }
        }
        it_seen = max_it_done;
    }
    HIP_TRY(hipEventRecord(ev1, s));
    if (int rc = batch_true_residual(B, nullptr)) return rc;
    for (int i = 0; i < nb; ++i)
        HIP_TRY(hipMemcpyAsync(u_out[i], B.probs[i]->u.p, B.probs[i]->hs.n * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    int first_bad = DDMGNN_OK;
    for (int i = 0; i < nb; ++i) {
        const KState& k = B.host_st[i];
        const bool converged = k.status == 0 && k.rel <= o.rtol;
        if (stats) {
            ddmgnn_stats& S = stats[i];
            std::memset(&S, 0, sizeof(S));
            S.iterations = k.it;
            S.converged = converged;
            S.rel_residual = k.rel;
            S.true_rel_residual = k.r0n > 0 ? std::sqrt(k.rr_true) / k.r0n : 0.0;
            S.solve_ms = ms;
            S.dss_launches = n_dss;
            S.dss_ms = t_dss;
            S.coarse_ms = t_coarse;
            S.prolong_ms = t_prolong;
            S.krylov_ms = t_krylov;
            S.dss_kernel = dss_kernel_of(B.probs[i], o);
            S.status = k.status ? k.status : (converged ? DDMGNN_OK : DDMGNN_E_MAXIT);
            S.latency_ms = ms;
        }
        if (first_bad == DDMGNN_OK) {
            if (k.status) first_bad = fail(k.status, "Krylov breakdown or non-finite residual");
            else if (!converged) first_bad = fail(DDMGNN_E_MAXIT, "not converged within max_it");
        }
    }
    return first_bad;
}

}  // namespace

// ------------------------------------------------------------------ batch API
void BatchDeleter::operator()(Batch* b) const { delete b; }

int build_batch(ddmgnn_ctx* ctx, ddmgnn_problem* const* probs, int n, BatchPtr& out) {
    BatchPtr B(new Batch());
    B->ctx = ctx;
    B->probs.assign(probs, probs + n);
    for (int i = 0; i < n; ++i) B->ids.push_back(probs[i]->id);
    B->model = probs[0]->model;
    struct W {
        int k, p, sub;
    };
    std::vector<W> all;
    std::vector<int2> vec, rows;
    for (int i = 0; i < n; ++i) {
        const ddmgnn_problem* P = probs[i];
        const auto& sp = P->hs.sub_ptr;
        for (int j = 0; j < P->hs.K; ++j) all.push_back({(int)(sp[j + 1] - sp[j]), i, j});
        const int nb = problem_vec_blocks(P);
        for (int b = 0; b < nb; ++b) vec.push_back(make_int2(i, b));
        for (int r = 0; r < P->hs.K; ++r) rows.push_back(make_int2(i, r));
    }
    // Largest sub-meshes first (a deterministic order: size, then problem, then sub-mesh).
    std::stable_sort(all.begin(), all.end(), [](const W& a, const W& b) {
        if (a.k != b.k) return a.k > b.k;
        if (a.p != b.p) return a.p < b.p;
        return a.sub < b.sub;
    });
    std::vector<int2> wa, wm, wms, wr, wv, wb;
    size_t lds_sb = 0, lds_db = 0, lds_small_sb = 0, lds_small_db = 0;
    for (const W& w : all) {
        wa.push_back(make_int2(w.p, w.sub));
        B->max_k_all = std::max(B->max_k_all, w.k);
        const ddmgnn_problem* Q = probs[w.p];
        if (w.k > kMaxSubNodes) {
            wb.push_back(make_int2(w.p, w.sub));
            continue;
        }
        wv.push_back(make_int2(w.p, w.sub));
        B->max_k_valu = std::max(B->max_k_valu, w.k);
        if (mfma_runs_sub(Q, w.sub)) {
            const size_t need = Q->mfma_need[w.sub];
            // Each launch reserves the largest need of its members; with two Q'
            // buffers where they fit that reserve (up to the kernel's limit, or
            // half a compute unit's LDS for the small workgroups), one otherwise.
            const size_t need_db = Q->mfma_need_db[w.sub];
            if (w.k <= MFMA_SMALL_K && need <= (size_t)Q->tune.small_lds) {
                wms.push_back(make_int2(w.p, w.sub));
                lds_small_sb = std::max(lds_small_sb, need);
                if (need_db <= MFMA_SMALL_LDS) lds_small_db = std::max(lds_small_db, need_db);
            } else {
                wm.push_back(make_int2(w.p, w.sub));
                lds_sb = std::max(lds_sb, need);
                if (need_db <= MFMA_LDS_LIMIT) lds_db = std::max(lds_db, need_db);
            }
        } else {
            wr.push_back(make_int2(w.p, w.sub));
            B->max_k_rest = std::max(B->max_k_rest, w.k);
        }
    }
    B->lds_mfma = std::max(lds_sb, lds_db);
    B->lds_mfma_small = std::max(lds_small_sb, lds_small_db);
    hipStream_t s = ctx->stream;
    if (int rc = upload_list(B->work_all, wa, s)) return rc;
    if (int rc = upload_list(B->work_mfma, wm, s)) return rc;
    if (int rc = upload_list(B->work_mfma_small, wms, s)) return rc;
    if (int rc = upload_list(B->work_rest, wr, s)) return rc;
    if (int rc = upload_list(B->work_valu, wv, s)) return rc;
    if (int rc = upload_list(B->work_big, wb, s)) return rc;
    if (int rc = upload_list(B->vec_blk, vec, s)) return rc;
    if (int rc = upload_list(B->coarse_rows, rows, s)) return rc;
    B->n_all = (int)wa.size();
    B->n_mfma = (int)wm.size();
    B->n_mfma_small = (int)wms.size();
    B->n_rest = (int)wr.size();
    B->n_valu = (int)wv.size();
    B->n_big = (int)wb.size();
    B->n_vec = (int)vec.size();
    B->n_coarse = (int)rows.size();
    HIP_TRY(B->st_gather.alloc(n));
    HIP_TRY(B->hook.alloc(1));
    HIP_TRY(hipHostMalloc((void**)&B->host_st, sizeof(KState) * n, hipHostMallocDefault));
    std::memset(B->host_st, 0, sizeof(KState) * n);
    if (int rc = upload_table(*B)) return rc;
    out = std::move(B);
    return DDMGNN_OK;
}

int batch_begin(Batch& B, const ddmgnn_solve_opts& o, const std::vector<uint8_t>* init) {
    bool changed = false;
    if (o.krylov != DDMGNN_CG && o.local_solver == DDMGNN_LOCAL_LU) {
        for (ddmgnn_problem* P : B.probs) {
            changed = changed || !P->lu_inv.p;
            if (int rc = prepare_lu(P)) return rc;
        }
    } else if (o.krylov != DDMGNN_CG) {
        if (int rc = prepare_dss(B, o.precision, changed)) return rc;
    }
    if (o.krylov == DDMGNN_FGMRES)
        if (int rc = prepare_fgmres(B, o.restart, changed)) return rc;
    if (changed && B.graph) {  // captured launches point at moved buffers
        (void)hipGraphExecDestroy(B.graph);
        B.graph = nullptr;
        B.graph_key = 0;
    }
    if (int rc = upload_table(B)) return rc;
    if (init) {
        if (int rc = upload_subset(B, init)) return rc;
        if (B.n_sub_blk)
            HIP_TRY(launch_init(B.tab.p, B.sub_blk.p, B.n_sub_blk, B.sub_list.p, B.n_sub_list, B.ctx->stream));
    }
    return DDMGNN_OK;
}

int batch_iterate(Batch& B, const ddmgnn_solve_opts& o, int count, bool use_graph) {
    if (use_graph) {
        if (!B.graph || B.graph_key != graph_key(o, count))
            if (int rc = capture_chunk(B, o, count)) return rc;
        HIP_TRY(hipGraphLaunch(B.graph, B.ctx->stream));
        return DDMGNN_OK;
    }
    for (int c = 0; c < count; ++c)
        if (int rc = enqueue_iteration(B, o, nullptr, false)) return rc;
    return DDMGNN_OK;
}

int batch_poll(Batch& B) {
    hipStream_t s = B.ctx->stream;
    const int n = (int)B.probs.size();
    HIP_TRY(launch_gather_states(B.tab.p, n, B.st_gather.p, s));
    HIP_TRY(hipMemcpyAsync(B.host_st, B.st_gather.p, sizeof(KState) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DDMGNN_OK;
}

const KState& batch_state(const Batch& B, int i) { return B.host_st[i]; }
int batch_size(const Batch& B) { return (int)B.probs.size(); }
ddmgnn_problem* batch_problem(const Batch& B, int i) { return B.probs[i]; }

int batch_true_residual(Batch& B, const std::vector<uint8_t>* which) {
    if (which) {
        if (int rc = upload_subset(B, which)) return rc;
        if (B.n_sub_blk)
            HIP_TRY(launch_resid(B.tab.p, B.sub_blk.p, B.n_sub_blk, B.sub_list.p, B.n_sub_list, B.ctx->stream));
    } else {
        HIP_TRY(launch_resid(B.tab.p, B.vec_blk.p, B.n_vec, nullptr, (int)B.probs.size(), B.ctx->stream));
    }
    return batch_poll(B);
}

int host_desc(const ddmgnn_problem_desc* in, HostDesc& h, const ddmgnn_problem_desc** out) {
    if (in->mem_kind == DDMGNN_MEM_HOST) {
        *out = in;
        return DDMGNN_OK;
    }
    if (in->mem_kind != DDMGNN_MEM_DEVICE) return fail(DDMGNN_E_INVALID, "mem_kind must be HOST or DEVICE");
    const int64_t n = in->n_nodes, nt = in->n_tri, K = in->n_sub;
    if (n <= 0 || nt <= 0 || K <= 0 || !in->a_rowptr || !in->sub_ptr)
        return fail(DDMGNN_E_INVALID, "empty problem");
    auto get = [&](auto& vec, const auto* src, int64_t count) -> hipError_t {
        if (!src || count <= 0) return hipSuccess;
        vec.resize((size_t)count);
        return hipMemcpy(vec.data(), src, (size_t)count * sizeof(vec[0]), hipMemcpyDeviceToHost);
    };
    HIP_TRY(get(h.a_rowptr, in->a_rowptr, n + 1));
    HIP_TRY(get(h.sub_ptr, in->sub_ptr, K + 1));
    const int64_t nnz = h.a_rowptr[n], sk = h.sub_ptr[K];
    if (nnz < 0 || sk < 0) return fail(DDMGNN_E_INVALID, "negative sizes");
    HIP_TRY(get(h.xy, in->xy, 2 * n));
    HIP_TRY(get(h.tri, in->tri, 3 * nt));
    HIP_TRY(get(h.dirichlet, in->dirichlet, n));
    HIP_TRY(get(h.a_col, in->a_col, nnz));
    HIP_TRY(get(h.a_val, in->a_val, nnz));
    HIP_TRY(get(h.b, in->b, n));
    HIP_TRY(get(h.u0, in->u0, n));
    HIP_TRY(get(h.sub_nodes, in->sub_nodes, sk));
    HIP_TRY(get(h.weights, in->weights, sk));
    auto ptr = [](auto& vec) { return vec.empty() ? nullptr : vec.data(); };
    ddmgnn_problem_desc& d = h.desc;
    d = *in;
    d.mem_kind = DDMGNN_MEM_HOST;
    d.xy = ptr(h.xy);
    d.tri = ptr(h.tri);
    d.dirichlet = ptr(h.dirichlet);
    d.a_rowptr = ptr(h.a_rowptr);
    d.a_col = ptr(h.a_col);
    d.a_val = ptr(h.a_val);
    d.b = ptr(h.b);
    d.u0 = ptr(h.u0);
    d.sub_ptr = ptr(h.sub_ptr);
    d.sub_nodes = ptr(h.sub_nodes);
    d.weights = ptr(h.weights);
    *out = &h.desc;
    return DDMGNN_OK;
}

int problem_vec_blocks(const ddmgnn_problem* P) {
    const int autom = vec_blocks(P->hs.n);
    return P->tune.vec_blocks > 0 ? std::min(autom, P->tune.vec_blocks) : autom;
}

// FGMRES storage for cycles of R steps: basis (R + 1) x n, Z R x n, partial sums
// (R + 1) x VEC_GRID, small arrays (H, rotations, g, y, tmp).
size_t fgmres_bytes(int64_t n, int R) {
    return 8 * ((size_t)(2 * R + 1) * n + (size_t)(R + 1) * VEC_GRID + (size_t)R * R + 6 * R + 2);
}

int dss_kernel_of(const ddmgnn_problem* P, const ddmgnn_solve_opts& o) {
    if (o.local_solver == DDMGNN_LOCAL_LU) return 3;
    if (o.precision == DDMGNN_FP64) return 0;
    if (o.precision != DDMGNN_BF16 || all_valu_bf16(P)) return 1;
    return any_valu_bf16(P) ? 4 : 2;
}

int check_opts(const ddmgnn_solve_opts& o) {
    if (o.krylov < 0 || o.krylov > 3) return fail(DDMGNN_E_INVALID, "krylov must be FCG, PCG, CG or FGMRES");
    if (o.krylov == DDMGNN_FGMRES && (o.restart < 1 || o.restart > MAX_RESTART))
        return fail(DDMGNN_E_INVALID, "restart must be in [1, 64]");
    if (o.krylov == DDMGNN_FCG && (o.m_max < 1 || o.m_max > MAX_M)) return fail(DDMGNN_E_INVALID, "m_max must be in [1, 4]");
    if (!(o.rtol >= 0.0)) return fail(DDMGNN_E_INVALID, "rtol must be >= 0");
    if (o.max_it < 0) return fail(DDMGNN_E_INVALID, "max_it must be >= 0");
    if (o.precision < 0 || o.precision > 2) return fail(DDMGNN_E_INVALID, "precision must be FP64, FP32 or BF16");
    if (o.prolong < 0 || o.prolong > 1) return fail(DDMGNN_E_INVALID, "prolong must be POU or UNWEIGHTED");
    if (o.local_solver < 0 || o.local_solver > 1) return fail(DDMGNN_E_INVALID, "local_solver must be GNN or LU");
    return DDMGNN_OK;
}

size_t problem_device_bytes(int64_t n, int64_t nnz, int32_t K, int64_t sk, int64_t ne) {
    size_t b = 0;
    b += 4 * (n + 1) + 12 * nnz;                 // CSR
    b += 8 * n * 2 + n;                          // b, u0, dirichlet
    b += 4 * (K + 1) + 12 * sk;                  // sub_ptr, sub_nodes, weights
    b += 4 * (sk + 1) + (2 + 4) * (ne + 8);      // edge_ptr, edge_src, edge_nd
    b += 4 * (ne + sk * (MFMA_EC - 1)) + 4 * (K + 1);  // padded edge records (bound), their ranges
    b += 16 * sk + 16 * sk + 8 * sk;             // tiles, xy64, xyc32
    b += 4 * (n + 1) + 8 * sk;                   // node_ptr, node_slots, slot_sub
    b += 8 * (size_t)K * K + 24 * (size_t)K;     // a0inv, s, y0, y
    b += 8 * sk;                                 // local
    b += 8 * n * (3 + 2 * (MAX_M + 1));          // u, r, z, direction ring
    b += 8 * (MAX_M + 1) * VEC_GRID + 16 + sizeof(KState);
    return b;
}

// The device-ready host arrays of a problem (HostSetup::upload_ready): plain
// host work, run by the caller of create_problem or by a server's setup worker.
std::string prepare_upload(const ddmgnn_problem_desc& desc, HostSetup& hs) {
    if (hs.upload_ready) return "";
    const int64_t n = hs.n, sk = hs.sk;
    const int K = hs.K;
    constexpr int64_t CH = 1 << 16;  // elements per task of the conversion loops
    hs.sp32.resize((size_t)K + 1);
    for (int i = 0; i <= K; ++i) hs.sp32[i] = (int32_t)desc.sub_ptr[i];
    hs.ep32.resize((size_t)sk + 1);
    hs.np32.resize((size_t)n + 1);
    hs.xy64.resize((size_t)2 * sk);
    hs.xyc32.resize((size_t)2 * sk);
    parallel_for((sk + CH) / CH, [&](int64_t c) {
        for (int64_t k = c * CH; k < std::min(sk + 1, (c + 1) * CH); ++k) hs.ep32[k] = (int32_t)hs.edge_ptr[k];
        for (int64_t k = c * CH; k < std::min(sk, (c + 1) * CH); ++k) {
            const int32_t v = desc.sub_nodes[k];
            hs.xy64[2 * k] = desc.xy[2 * v];
            hs.xy64[2 * k + 1] = desc.xy[2 * v + 1];
            hs.xyc32[2 * k] = (float)hs.xyc[2 * k];
            hs.xyc32[2 * k + 1] = (float)hs.xyc[2 * k + 1];
        }
    });
    parallel_for((n + CH) / CH, [&](int64_t c) {
        for (int64_t i = c * CH; i < std::min(n + 1, (c + 1) * CH); ++i) hs.np32[i] = (int32_t)hs.node_ptr[i];
    });
    // padded by 8 entries: the chunked edge loops read up to 3 past a node's last edge
    hs.src_pad.assign(hs.edge_src.begin(), hs.edge_src.end());
    hs.src_pad.resize(hs.src_pad.size() + 8, 0);
    hs.nd_pad.assign(hs.edge_nd.begin(), hs.edge_nd.end());
    hs.nd_pad.resize(hs.nd_pad.size() + 8, 0.0f);
    // MFMA kernel records, per tile of MFMA_TILE nodes (tile order): slot-major
    // [slot][lane] blocks padded with sentinel records (sender k_i, |d| 0)
    // to the tile's largest in-degree rounded up to MFMA_EC. Tile records
    // hold the block's offset in the sub-mesh (low 24 bits) and its number
    // of MFMA_EC-slot chunks (high 8 bits). Sub-meshes are independent: the
    // sizes of their edge blocks first, then their records in parallel.
    hs.mfma_need.assign(K, 0);
    hs.mfma_need_db.assign(K, 0);
    std::vector<int64_t> esize((size_t)K, 0);
    std::atomic<int> too_big{0};
    parallel_for(K, [&](int64_t i) {
        const int64_t b = desc.sub_ptr[i], k = desc.sub_ptr[i + 1] - b;
        if (k > kMaxSubNodes) return;  // the VALU kernel's global-memory form runs it: no tile records
        int64_t size = 0;
        for (int64_t t0 = 0; t0 < k; t0 += MFMA_TILE) {
            int maxdeg = 0;
            for (int64_t q = t0; q < std::min<int64_t>(k, t0 + MFMA_TILE); ++q) {
                const int64_t slot = b + hs.tnode[b + q];
                maxdeg = std::max<int>(maxdeg, (int)(hs.edge_ptr[slot + 1] - hs.edge_ptr[slot]));
            }
            const int nch = (maxdeg + MFMA_EC - 1) / MFMA_EC;
            if (nch > 255 || size + (int64_t)nch * MFMA_EC * MFMA_TILE >= (1 << 24)) too_big = 1;
            size += (int64_t)nch * MFMA_EC * MFMA_TILE;
        }
        esize[i] = size;
    });
    if (too_big) return "sub-mesh edge block too large for the MFMA tile records";
    std::vector<int32_t>& epad = hs.mfma_epad;
    epad.assign((size_t)K + 1, 0);
    for (int i = 0; i < K; ++i) {
        if (epad[i] + esize[i] >= INT32_MAX) return "edge records beyond 32-bit offsets";
        epad[i + 1] = (int32_t)(epad[i] + esize[i]);
    }
    std::vector<uint32_t>& er = hs.mfma_erec;
    er.assign((size_t)epad[K], 0u);
    hs.has_big = false;
    std::vector<TileNode> tiles(sk);
    parallel_for(K, [&](int64_t i) {
        const int64_t b = desc.sub_ptr[i], e = desc.sub_ptr[i + 1];
        const int k = (int)(e - b);
        if (k > kMaxSubNodes) {
            hs.mfma_need[i] = UINT32_MAX;
            hs.mfma_need_db[i] = UINT32_MAX;
            return;
        }
        std::vector<int64_t> cand;  // per lane of a tile: its in-edges, in order
        std::vector<uint8_t> taken;
        size_t off = 0;
        for (int t0 = 0; t0 < k; t0 += MFMA_TILE) {
            const int t1 = std::min(k, t0 + MFMA_TILE);
            int maxdeg = 0;
            for (int q = t0; q < t1; ++q) {
                const int64_t slot = b + hs.tnode[b + q];
                maxdeg = std::max<int>(maxdeg, (int)(hs.edge_ptr[slot + 1] - hs.edge_ptr[slot]));
            }
            const int nch = (maxdeg + MFMA_EC - 1) / MFMA_EC;
            uint32_t* blk = er.data() + epad[i] + off;
            std::fill(blk, blk + (size_t)nch * MFMA_EC * MFMA_TILE, mfma_edge_record(k, 0));
            // Slot by slot, each lane takes the first remaining in-edge whose sender
            // row starts on the least used LDS bank of the slot (rows are 5 dwords
            // apart), so a wavefront's gathers spread over the banks. This only
            // reorders each node's message sum.
            cand.assign((size_t)(t1 - t0) * maxdeg, -1);
            taken.assign(cand.size(), 0);
            for (int q = t0; q < t1; ++q) {
                const int64_t slot = b + hs.tnode[b + q];
                for (int64_t t = hs.edge_ptr[slot]; t < hs.edge_ptr[slot + 1]; ++t)
                    cand[(size_t)(q - t0) * maxdeg + (t - hs.edge_ptr[slot])] = t;
            }
            for (int w = 0; w < maxdeg; ++w) {
                int used[32] = {0};
                for (int q = t0; q < t1; ++q) {
                    const int64_t* c = cand.data() + (size_t)(q - t0) * maxdeg;
                    uint8_t* tk = taken.data() + (size_t)(q - t0) * maxdeg;
                    int best = -1;
                    for (int x = 0; x < maxdeg && c[x] >= 0; ++x)
                        if (!tk[x] && (best < 0 || used[(5 * hs.edge_src[c[x]]) % 32] <
                                                       used[(5 * hs.edge_src[c[best]]) % 32]))
                            best = x;
                    if (best < 0) continue;
                    const int64_t t = c[best];
                    tk[best] = 1;
                    used[(5 * hs.edge_src[t]) % 32]++;
                    blk[(size_t)w * MFMA_TILE + (q - t0)] = mfma_edge_record(hs.edge_src[t], (uint16_t)(hs.erec[t] >> 16));
                }
            }
            for (int q = t0; q < t1; ++q) {
                const int32_t j = hs.tnode[b + q];
                const int64_t slot = b + j;
                TileNode& tn = tiles[b + q];
                tn.e0 = (int32_t)((uint32_t)off | ((uint32_t)nch << 24));
                tn.j = (uint16_t)j;
                tn.deg = (uint16_t)(hs.edge_ptr[slot + 1] - hs.edge_ptr[slot]);
                tn.xh = hs.xyhl[4 * slot + 0];
                tn.xl = hs.xyhl[4 * slot + 1];
                tn.yh = hs.xyhl[4 * slot + 2];
                tn.yl = hs.xyhl[4 * slot + 3];
            }
            off += (size_t)nch * MFMA_EC * MFMA_TILE;
        }
        hs.mfma_need[i] = (uint32_t)mfma_lds_need(k, esize[i]);
        hs.mfma_need_db[i] = (uint32_t)mfma_lds_need(k, esize[i], true);
    });
    for (int i = 0; i < K; ++i) hs.has_big = hs.has_big || hs.mfma_need[i] == UINT32_MAX;
    static_assert(sizeof(TileNode) == 4 * sizeof(uint32_t), "tile records are four words");
    hs.mfma_tiles.resize((size_t)4 * sk);
    if (sk) std::memcpy(hs.mfma_tiles.data(), tiles.data(), (size_t)sk * sizeof(TileNode));
    hs.upload_ready = true;
    return "";
}

int create_problem(ddmgnn_ctx* ctx, const ddmgnn_problem_desc& desc, std::shared_ptr<ModelDev> model,
                   HostSetup&& hs_in, ddmgnn_problem** out, hipStream_t stream) {
    auto P = std::make_unique<ddmgnn_problem>();
    P->ctx = ctx;
    P->id = g_next_id.fetch_add(1);
    P->hs = std::move(hs_in);
    P->model = std::move(model);
    {
        const std::string e = prepare_upload(desc, P->hs);
        if (!e.empty()) return fail(DDMGNN_E_INVALID, e);
    }
    const auto& hs = P->hs;
    const int64_t n = hs.n, sk = hs.sk;
    const int K = hs.K;
    hipStream_t s = stream ? stream : ctx->stream;
    HIP_TRY(P->rowptr.upload(desc.a_rowptr, n + 1, s));
    HIP_TRY(P->col.upload(desc.a_col, hs.nnz, s));
    HIP_TRY(P->val.upload(desc.a_val, hs.nnz, s));
    HIP_TRY(P->b.upload(desc.b, n, s));
    HIP_TRY(P->u0.upload(desc.u0, n, s));
    HIP_TRY(P->dirichlet.upload(desc.dirichlet, n, s));
    HIP_TRY(P->sub_ptr.upload(hs.sp32.data(), K + 1, s));
    HIP_TRY(P->sub_nodes.upload(desc.sub_nodes, sk, s));
    HIP_TRY(P->weights.upload(desc.weights, sk, s));
    HIP_TRY(P->edge_ptr.upload(hs.ep32.data(), sk + 1, s));
    HIP_TRY(P->edge_src.upload(hs.src_pad.data(), hs.src_pad.size(), s));
    HIP_TRY(P->node_ptr.upload(hs.np32.data(), n + 1, s));
    HIP_TRY(P->node_slots.upload(hs.node_slots.data(), sk, s));
    HIP_TRY(P->slot_sub.upload(hs.slot_sub.data(), sk, s));
    HIP_TRY(P->xy64.upload(hs.xy64.data(), 2 * sk, s));
    HIP_TRY(P->xyc32.upload(hs.xyc32.data(), 2 * sk, s));
    if (!hs.a0inv.empty()) {
        HIP_TRY(P->a0inv.upload(hs.a0inv.data(), (size_t)K * K, s));
    } else {  // the coarse operator and its inverse, formed on the device
        const int64_t off_h[2] = {0, (int64_t)K * K};
        HIP_TRY(P->a0inv.alloc((size_t)K * K));
        HIP_TRY(P->coarse_diag0.alloc((size_t)K));
        HIP_TRY(P->coarse_off.upload(off_h, 2, s));
        HIP_TRY(launch_coarse_assemble(P->rowptr.p, P->col.p, P->val.p, P->sub_ptr.p, P->sub_nodes.p, P->weights.p,
                                       P->node_ptr.p, P->node_slots.p, P->slot_sub.p, K, P->a0inv.p,
                                       P->coarse_diag0.p, s));
        const int rc = gj_invert_batch(std::vector<int32_t>{K}, P->a0inv.p, P->coarse_off.p, P->coarse_diag0.p, s,
                                       P->coarse_gj);
        if (rc == DDMGNN_E_NOT_SPD) return fail(rc, "coarse matrix R_0 A R_0^T is not positive definite");
        if (rc) return rc;
    }
    if (!hs.lu_inv.empty()) {
        HIP_TRY(P->lu_off.upload(hs.lu_off.data(), hs.lu_off.size(), s));
        HIP_TRY(P->lu_inv.upload(hs.lu_inv.data(), hs.lu_inv.size(), s));
    }
    P->mfma_need = hs.mfma_need;
    P->mfma_need_db = hs.mfma_need_db;
    P->has_big = hs.has_big;
    HIP_TRY(P->tiles.upload(reinterpret_cast<const TileNode*>(hs.mfma_tiles.data()), (size_t)sk, s));
    HIP_TRY(P->erec.upload(hs.mfma_erec.data(), std::max<size_t>(hs.mfma_erec.size(), 1), s));
    HIP_TRY(P->epad_sub.upload(hs.mfma_epad.data(), hs.mfma_epad.size(), s));
    HIP_TRY(P->edge_nd.upload(hs.nd_pad.data(), hs.nd_pad.size(), s));
    HIP_TRY(P->s.alloc(K));
    HIP_TRY(P->y0.alloc(K));
    HIP_TRY(P->y.alloc(K));
    HIP_TRY(P->local.alloc(sk));
    HIP_TRY(P->u.alloc(n));
    HIP_TRY(P->r.alloc(n));
    HIP_TRY(P->z.alloc(n));
    HIP_TRY(P->ring.alloc((size_t)2 * (MAX_M + 1) * n));
    HIP_TRY(P->st.alloc(1));
    HIP_TRY(P->partials.alloc((size_t)(MAX_M + 1) * VEC_GRID));
    HIP_TRY(hipMemsetAsync(P->st.p, 0, sizeof(KState), s));
    HIP_TRY(hipStreamSynchronize(s));
    P->device_bytes = problem_device_bytes(n, hs.nnz, K, sk, hs.n_edges) + P->lu_inv.n * sizeof(double) +
                      P->lu_off.n * sizeof(int64_t);
    // host copies of the uploaded arrays are not needed again
    std::vector<double>().swap(P->hs.lu_inv);
    std::vector<int64_t>().swap(P->hs.lu_off);
    HostSetup& h = P->hs;
    std::vector<int32_t>().swap(h.sp32);
    std::vector<int32_t>().swap(h.ep32);
    std::vector<int32_t>().swap(h.np32);
    std::vector<double>().swap(h.xy64);
    std::vector<float>().swap(h.xyc32);
    std::vector<float>().swap(h.nd_pad);
    std::vector<uint16_t>().swap(h.src_pad);
    std::vector<uint32_t>().swap(h.mfma_erec);
    std::vector<uint32_t>().swap(h.mfma_tiles);
    std::vector<int32_t>().swap(h.mfma_epad);
    h.upload_ready = false;
    *out = P.release();
    return DDMGNN_OK;
}

}  // namespace ddmgnn

using namespace ddmgnn;

ddmgnn_ctx::~ddmgnn_ctx() {
    last_batch.reset();
    if (host_pinned) (void)hipHostFree(host_pinned);
    if (cap) (void)hipStreamDestroy(cap);
    if (side) (void)hipStreamDestroy(side);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
}

// Drops the cached batches that hold P (its own and the context's last one).
void drop_batches(ddmgnn_problem* P) {
    P->solo.reset();
    if (P->ctx && P->ctx->last_batch) {
        const auto& B = *P->ctx->last_batch;
        if (std::find(B.ids.begin(), B.ids.end(), P->id) != B.ids.end()) P->ctx->last_batch.reset();
    }
}

ddmgnn_problem::~ddmgnn_problem() { drop_batches(this); }

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* ddmgnn_last_error(void) { return g_err.c_str(); }
const char* ddmgnn_version(void) { return "ddmgnn 0.2 gfx950"; }
int32_t ddmgnn_max_subdomain_nodes(void) { return kMaxSubNodesAny; }

void ddmgnn_default_opts(ddmgnn_solve_opts* o) {
    o->krylov = DDMGNN_FCG;
    o->m_max = 1;
    o->rtol = 1e-6;
    o->max_it = 10000;
    o->precision = DDMGNN_FP32;
    o->prolong = DDMGNN_PROLONG_POU;
    o->coarse = 1;
    o->check_every = 16;
    o->profile = 0;
    o->graph = 1;
    o->local_solver = DDMGNN_LOCAL_GNN;
    o->restart = 30;
}

int ddmgnn_ctx_create(void* hip_stream, ddmgnn_ctx** out) {
    if (!out) return fail(DDMGNN_E_INVALID, "null output pointer");
    auto c = std::make_unique<ddmgnn_ctx>();
    c->stream = (hipStream_t)hip_stream;
    c->launch = c->stream;
    HIP_TRY(hipGetDevice(&c->device));
    HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    HIP_TRY(c->partials.alloc(VEC_GRID));
    HIP_TRY(c->scalar.alloc(1));
    HIP_TRY(hipHostMalloc((void**)&c->host_pinned, 256, hipHostMallocDefault));
    HIP_TRY(noalloc_init(c->device));  // with the context's device current
    *out = c.release();
    return DDMGNN_OK;
}

int ddmgnn_ctx_destroy(ddmgnn_ctx* ctx) {
    delete ctx;
    return DDMGNN_OK;
}

int ddmgnn_model_create(ddmgnn_ctx* ctx, const ddmgnn_model_desc* desc, const float* theta, int64_t n_theta,
                        ddmgnn_model** out) {
    if (!ctx || !desc || !theta || !out) return fail(DDMGNN_E_INVALID, "null argument");
    const int d = desc->d;
    if (d != 5 && d != 10 && d != 20) return fail(DDMGNN_E_INVALID, "latent width d must be 5, 10 or 20");
    if (desc->kbar < 1) return fail(DDMGNN_E_INVALID, "kbar must be >= 1");
    const int64_t expect = (int64_t)desc->kbar * (11 * d * d + 15 * d + 1);
    if (n_theta != expect) return fail(DDMGNN_E_INVALID, "n_theta must equal kbar*(11d^2+15d+1)");
    for (int64_t i = 0; i < n_theta; ++i)
        if (!std::isfinite(theta[i])) return fail(DDMGNN_E_INVALID, "non-finite weight");
    auto m = std::make_unique<ddmgnn_model>();
    m->kbar = desc->kbar;
    m->d = desc->d;
    m->alpha = desc->alpha;
    m->theta.assign(theta, theta + n_theta);
    std::vector<MfmaStep> steps;
    std::vector<MfmaDec> dec;
    if (d == D) {
        build_mfma_blobs(m->theta.data(), m->kbar, steps, dec);
    } else if (d < D) {  // the matrix-core kernel runs the model embedded in width 10
        std::vector<float> padded;
        pad_theta_to_d10(m->theta.data(), m->kbar, d, padded);
        build_mfma_blobs(padded.data(), m->kbar, steps, dec);
    }
    auto dev = std::make_shared<ModelDev>();
    dev->id = g_next_id.fetch_add(1);
    dev->kbar = m->kbar;
    dev->d = d;
    dev->mfma = d <= D;
    dev->alpha = m->alpha;
    hipStream_t s = ctx->stream;
    std::vector<double> th64(m->theta.begin(), m->theta.end());
    HIP_TRY(dev->theta32.upload(m->theta.data(), m->theta.size(), s));
    HIP_TRY(dev->theta64.upload(th64.data(), th64.size(), s));
    HIP_TRY(dev->steps.upload(steps.data(), steps.size(), s));
    HIP_TRY(dev->dec.upload(dec.data(), dec.size(), s));
    m->dev = std::move(dev);
    *out = m.release();
    return DDMGNN_OK;
}

int ddmgnn_model_init_xavier(const ddmgnn_model_desc* desc, uint64_t seed, float* theta, int64_t n_theta) {
    if (!desc || !theta) return fail(DDMGNN_E_INVALID, "null argument");
    const int64_t d = desc->d, kbar = desc->kbar;
    if (d < 1 || kbar < 1 || n_theta != kbar * (11 * d * d + 15 * d + 1))
        return fail(DDMGNN_E_INVALID, "n_theta must equal kbar*(11d^2+15d+1)");
    uint64_t state = seed;
    auto next = [&]() {  // splitmix64
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    int64_t pos = 0;
    auto layer = [&](int64_t fan_out, int64_t fan_in) {
        const double a = std::sqrt(6.0 / (double)(fan_in + fan_out));
        for (int64_t i = 0; i < fan_out * fan_in; ++i) {
            const double u = (double)(next() >> 11) * 0x1.0p-53;
            theta[pos++] = (float)(a * (2.0 * u - 1.0));
        }
        for (int64_t i = 0; i < fan_out; ++i) theta[pos++] = 0.0f;
    };
    for (int64_t k = 0; k < kbar; ++k) {
        for (int phi = 0; phi < 2; ++phi) {
            layer(d, 2 * d + 3);
            layer(d, d);
        }
        layer(d, 3 * d + 1);
        layer(d, d);
        layer(d, d);
        layer(1, d);
    }
    return DDMGNN_OK;
}

int ddmgnn_model_destroy(ddmgnn_model* m) {
    delete m;
    return DDMGNN_OK;
}

int ddmgnn_validate_problem(const ddmgnn_problem_desc* desc_in) {
    if (!desc_in) return fail(DDMGNN_E_INVALID, "null descriptor");
    HostDesc hd;
    const ddmgnn_problem_desc* desc = nullptr;
    if (int rc = host_desc(desc_in, hd, &desc)) return rc;
    std::string e = validate(*desc);
    if (!e.empty()) return fail(DDMGNN_E_INVALID, e);
    return DDMGNN_OK;
}

int ddmgnn_problem_create(ddmgnn_ctx* ctx, const ddmgnn_problem_desc* desc_in, const ddmgnn_model* model,
                          ddmgnn_problem** out) {
    if (!ctx || !desc_in || !model || !out) return fail(DDMGNN_E_INVALID, "null argument");
    HostDesc hd;
    const ddmgnn_problem_desc* desc = nullptr;
    if (int rc = host_desc(desc_in, hd, &desc)) return rc;
    int rc = ddmgnn_validate_problem(desc);
    if (rc) return rc;
    HostSetup hs;
    std::string e = build_setup(*desc, hs, false);  // the coarse level is formed on the device
    if (!e.empty()) return fail(DDMGNN_E_INVALID, e);
    return create_problem(ctx, *desc, model->dev, std::move(hs), out);
}

int ddmgnn_problem_destroy(ddmgnn_problem* P) {
    delete P;
    return DDMGNN_OK;
}

int ddmgnn_problem_sizes(const ddmgnn_problem* P, int64_t* n, int64_t* nnz, int32_t* k, int64_t* sum_k,
                         int64_t* n_edges) {
    if (!P) return fail(DDMGNN_E_INVALID, "null problem");
    if (n) *n = P->hs.n;
    if (nnz) *nnz = P->hs.nnz;
    if (k) *k = P->hs.K;
    if (sum_k) *sum_k = P->hs.sk;
    if (n_edges) *n_edges = P->hs.n_edges;
    return DDMGNN_OK;
}

int ddmgnn_problem_set_tuning(ddmgnn_problem* P, const ddmgnn_tuning* t) {
    if (!P || !t) return fail(DDMGNN_E_INVALID, "null argument");
    if (t->small_lds < 0 || t->small_lds > (int32_t)MFMA_SMALL_LDS)
        return fail(DDMGNN_E_INVALID, "small_lds must be in [0, 80 KiB - 1 KiB]");
    if (t->vec_blocks != 0 && (t->vec_blocks < N_XCD || t->vec_blocks > VEC_GRID || t->vec_blocks % N_XCD))
        return fail(DDMGNN_E_INVALID, "vec_blocks must be 0 or a multiple of 8 in [8, 1024]");
    if (t->small_lds != P->tune.small_lds || t->vec_blocks != P->tune.vec_blocks) {
        P->tune = *t;
        drop_batches(P);
    }
    return DDMGNN_OK;
}

int ddmgnn_problem_get_tuning(const ddmgnn_problem* P, ddmgnn_tuning* t) {
    if (!P || !t) return fail(DDMGNN_E_INVALID, "null argument");
    *t = P->tune;
    return DDMGNN_OK;
}

int ddmgnn_autotune(ddmgnn_ctx* ctx, ddmgnn_problem* P, const ddmgnn_solve_opts* opts, int32_t iterations,
                    ddmgnn_tuning* best, double* ms_per_iteration) {
    if (!ctx || !P || !opts) return fail(DDMGNN_E_INVALID, "null argument");
    if (iterations < 1) return fail(DDMGNN_E_INVALID, "iterations must be >= 1");
    if (int rc = check_opts(*opts)) return rc;
    ddmgnn_solve_opts o = *opts;
    o.max_it = iterations;
    o.rtol = 0.0;  // run the capped number of iterations
    o.graph = 1;
    o.profile = 0;
    o.check_every = std::min(iterations, 16);
    // time per iteration of a candidate: best of two capped solves (the first of a
    // schedule also captures its graph)
    auto timed = [&](const ddmgnn_tuning& t, double& ms) -> int {
        if (int rc = ddmgnn_problem_set_tuning(P, &t)) return rc;
        if (int rc = solo_batch(P)) return rc;
        double best_ms = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            ddmgnn_stats st{};
            double* outs[1] = {P->z.p};  // the solution copy lands in scratch
            const int rc = solve_batch(ctx, *P->solo, o, outs, &st);
            if (rc && rc != DDMGNN_E_MAXIT) return rc;
            if (rep > 0) best_ms = std::min(best_ms, st.solve_ms / std::max(1, st.iterations));
        }
        ms = best_ms;
        return DDMGNN_OK;
    };
    const bool mfma = o.krylov != DDMGNN_CG && o.local_solver == DDMGNN_LOCAL_GNN &&
                      dss_kernel_of(P, o) == 2;
    ddmgnn_tuning cur{0, 0}, top{0, 0};
    double top_ms = 1e300;
    std::vector<int32_t> lds = {0};
    if (mfma) lds = {0, 48 * 1024, 64 * 1024, (int32_t)MFMA_SMALL_LDS};
    for (int32_t v : lds) {
        cur.small_lds = v;
        double ms = 0;
        if (int rc = timed(cur, ms)) return rc;
        if (ms < top_ms) {
            top_ms = ms;
            top = cur;
        }
    }
    cur = top;
    for (int32_t vb : {256, 512, 1024}) {
        if (vb > vec_blocks(P->hs.n)) continue;
        cur.vec_blocks = vb;
        double ms = 0;
        if (int rc = timed(cur, ms)) return rc;
        if (ms < top_ms) {
            top_ms = ms;
            top = cur;
        }
    }
    if (int rc = ddmgnn_problem_set_tuning(P, &top)) return rc;
    if (best) *best = top;
    if (ms_per_iteration) *ms_per_iteration = top_ms;
    return DDMGNN_OK;
}

int ddmgnn_problem_device_bytes(const ddmgnn_problem* P, int64_t* bytes) {
    if (!P || !bytes) return fail(DDMGNN_E_INVALID, "null argument");
    *bytes = (int64_t)P->device_bytes;
    return DDMGNN_OK;
}

int ddmgnn_setup_local_graph(const ddmgnn_problem_desc* desc_in, int32_t sub, int32_t* rowptr, int32_t* col,
                             int64_t* n_edges_sub) {
    if (!desc_in) return fail(DDMGNN_E_INVALID, "null descriptor");
    HostDesc hd;
    const ddmgnn_problem_desc* desc = nullptr;
    if (int rc = host_desc(desc_in, hd, &desc)) return rc;
    int rc = ddmgnn_validate_problem(desc);
    if (rc) return rc;
    if (sub < 0 || sub >= desc->n_sub) return fail(DDMGNN_E_INVALID, "sub-mesh index out of range");
    HostSetup hs;
    build_local_graphs(*desc, hs);
    const int64_t b = desc->sub_ptr[sub], e = desc->sub_ptr[sub + 1];
    const int64_t e0 = hs.edge_ptr[b], e1 = hs.edge_ptr[e];
    if (n_edges_sub) *n_edges_sub = e1 - e0;
    if (rowptr)
        for (int64_t k = b; k <= e; ++k) rowptr[k - b] = (int32_t)(hs.edge_ptr[k] - e0);
    if (col)
        for (int64_t q = e0; q < e1; ++q) col[q - e0] = hs.edge_src[q];
    return DDMGNN_OK;
}

int ddmgnn_setup_coarse(const ddmgnn_problem_desc* desc_in, double* a0, double* a0inv) {
    if (!desc_in) return fail(DDMGNN_E_INVALID, "null descriptor");
    HostDesc hd;
    const ddmgnn_problem_desc* desc = nullptr;
    if (int rc = host_desc(desc_in, hd, &desc)) return rc;
    int rc = ddmgnn_validate_problem(desc);
    if (rc) return rc;
    HostSetup hs;
    std::string e = build_setup(*desc, hs);
    if (!hs.a0.empty() && a0) std::memcpy(a0, hs.a0.data(), hs.a0.size() * sizeof(double));
    if (e == "NOT_SPD") return fail(DDMGNN_E_NOT_SPD, "coarse matrix R_0 A R_0^T is not positive definite");
    if (!e.empty()) return fail(DDMGNN_E_INVALID, e);
    if (a0inv) std::memcpy(a0inv, hs.a0inv.data(), hs.a0inv.size() * sizeof(double));
    return DDMGNN_OK;
}

int ddmgnn_setup_local_inverse(const ddmgnn_problem_desc* desc_in, int32_t sub, double* inv) {
    if (!desc_in) return fail(DDMGNN_E_INVALID, "null descriptor");
    HostDesc hd;
    const ddmgnn_problem_desc* desc = nullptr;
    if (int rc = host_desc(desc_in, hd, &desc)) return rc;
    int rc = ddmgnn_validate_problem(desc);
    if (rc) return rc;
    if (sub < 0 || sub >= desc->n_sub || !inv) return fail(DDMGNN_E_INVALID, "sub-mesh index out of range or null output");
    std::vector<double> m;
    if (!local_inverse(*desc, sub, m, true).empty())
        return fail(DDMGNN_E_NOT_SPD, "local matrix R_i A R_i^T is not positive definite");
    std::memcpy(inv, m.data(), m.size() * sizeof(double));
    return DDMGNN_OK;
}

int ddmgnn_spmv(ddmgnn_ctx* ctx, ddmgnn_problem* P, const double* x, double* y) {
    if (!ctx || !P || !x || !y) return fail(DDMGNN_E_INVALID, "null argument");
    HIP_TRY(launch_spmv(P->rowptr.p, P->col.p, P->val.p, x, y, (int)P->hs.n, problem_vec_blocks(P), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DDMGNN_OK;
}

int ddmgnn_dot(ddmgnn_ctx* ctx, int64_t n, const double* x, const double* y, double* out) {
    if (!ctx || !out || n < 0 || n > INT32_MAX || (n > 0 && (!x || !y))) return fail(DDMGNN_E_INVALID, "invalid argument");
    if (n == 0) {
        *out = 0.0;
        return DDMGNN_OK;
    }
    HIP_TRY(launch_dot(x, y, (int)n, ctx->partials.p, ctx->scalar.p, ctx->stream, true));
    HIP_TRY(hipMemcpyAsync(ctx->host_pinned, ctx->scalar.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *out = ctx->host_pinned[0];
    return DDMGNN_OK;
}

int ddmgnn_dot_noalloc(ddmgnn_ctx* ctx, int64_t n, const double* x, const double* y, double* out) {
    if (!ctx || !out || n < 0 || (n > 0 && (!x || !y))) return fail(DDMGNN_E_INVALID, "null argument or n < 0");
    if (n > DDMGNN_NOALLOC_DOT_MAX_N)
        return fail(DDMGNN_E_INVALID, "ddmgnn_dot_noalloc: n exceeds DDMGNN_NOALLOC_DOT_MAX_N (2^31 - 1)");
    double* scr = noalloc_scratch(ctx->device);
    if (!scr) return fail(DDMGNN_E_INVALID, "ddmgnn_dot_noalloc: no scratch address for the context's device");
    // n = 0 runs the same kernels over no rows: the partials are 0 and so is *out.
    HIP_TRY(launch_dot(x, y, (int)n, scr, out, ctx->stream, true));
    return DDMGNN_OK;
}

int ddmgnn_dss_forward(ddmgnn_ctx* ctx, ddmgnn_problem* P, int32_t precision, const double* c, double* out) {
    if (!ctx || !P || !c || !out) return fail(DDMGNN_E_INVALID, "null argument");
    if (precision < 0 || precision > 2) return fail(DDMGNN_E_INVALID, "bad precision");
    if (int rc = solo_batch(P)) return rc;
    Batch& B = *P->solo;
    bool changed = false;
    if (int rc = prepare_dss(B, precision, changed)) return rc;
    DevProb v = make_view(P);
    v.c_in = c;
    v.local = out;
    v.st = nullptr;
    HIP_TRY(upload_async(B.hook.p, &v, sizeof(v), ctx->stream));
    if (int rc = enqueue_dss(B, B.hook.p, precision, 0, false)) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DDMGNN_OK;
}

int ddmgnn_dss_forward_sub(ddmgnn_ctx* ctx, ddmgnn_problem* P, int32_t precision, int32_t sub, const double* c,
                           double* out) {
    if (!ctx || !P || !c || !out) return fail(DDMGNN_E_INVALID, "null argument");
    if (precision < 0 || precision > 2) return fail(DDMGNN_E_INVALID, "bad precision");
    if (sub < 0 || sub >= P->hs.K) return fail(DDMGNN_E_INVALID, "sub-mesh index out of range");
    if (int rc = solo_batch(P)) return rc;
    Batch& B = *P->solo;
    bool changed = false;
    if (int rc = prepare_dss(B, precision, changed)) return rc;
    hipStream_t s = ctx->stream;
    const int64_t base = P->hs.sub_ptr[sub], k = P->hs.sub_ptr[sub + 1] - base;
    if (!P->fwd_in.p) {
        HIP_TRY(P->fwd_in.alloc((size_t)P->hs.sk));
        HIP_TRY(P->fwd_out.alloc((size_t)P->hs.sk));
        HIP_TRY(P->one_work.alloc(1));
    }
    const int2 item = make_int2(0, sub);
    HIP_TRY(upload_async(P->one_work.p, &item, sizeof(item), s));
    HIP_TRY(hipMemcpyAsync(P->fwd_in.p + base, c, (size_t)k * sizeof(double), hipMemcpyDeviceToDevice, s));
    DevProb v = make_view(P);
    v.c_in = P->fwd_in.p;
    v.local = P->fwd_out.p;
    v.st = nullptr;
    HIP_TRY(upload_async(B.hook.p, &v, sizeof(v), s));
    const ModelDev& M = *B.model;
    const int vprec = precision == DDMGNN_BF16 ? DDMGNN_FP32 : precision;
    if (k > kMaxSubNodes) {
        HIP_TRY(launch_dss_big(B.hook.p, P->one_work.p, 1, vprec, M.d, M.kbar, M.alpha, 0, M.theta32.p,
                               M.theta64.p, s, true));
    } else if (precision == DDMGNN_BF16 && mfma_runs_sub(P, sub)) {
        DssMfmaArgs a{B.hook.p, P->one_work.p, M.steps.p, M.dec.p, M.kbar, (float)M.alpha, 0};
        const size_t shmem = P->mfma_need_db[sub] <= MFMA_LDS_LIMIT ? P->mfma_need_db[sub] : P->mfma_need[sub];
        HIP_TRY(launch_dss_mfma(a, 1, shmem, MFMA_BLOCK, s, true));
    } else {
        const int mk = precision == DDMGNN_BF16 ? B.max_k_rest : B.max_k_valu;  // as prepare_dss sized it
        const bool qlds = valu_q_in_lds(mk, vprec, M.d);
        HIP_TRY(launch_dss_valu(B.hook.p, P->one_work.p, 1, vprec, M.d, qlds, M.kbar, M.alpha, 0, M.theta32.p,
                                M.theta64.p, qlds ? valu_shmem(mk, vprec, M.d) : 0, s, true));
    }
    HIP_TRY(hipMemcpyAsync(out, P->fwd_out.p + base, (size_t)k * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DDMGNN_OK;
}

int ddmgnn_time_apply_stages(ddmgnn_ctx* ctx, ddmgnn_problem* P, const ddmgnn_solve_opts* opts, const double* r,
                             double* z, int32_t reps, double* local_ms, double* coarse_ms, double* glue_ms) {
    if (!ctx || !P || !opts || !r || !z) return fail(DDMGNN_E_INVALID, "null argument");
    if (r == z) return fail(DDMGNN_E_INVALID, "r and z must not alias");
    if (reps < 1) return fail(DDMGNN_E_INVALID, "reps must be >= 1");
    if (int rc = check_opts(*opts)) return rc;
    if (int rc = solo_batch(P)) return rc;
    Batch& B = *P->solo;
    bool changed = false;
    if (opts->local_solver == DDMGNN_LOCAL_LU) {
        if (int rc = prepare_lu(P)) return rc;
    } else if (int rc = prepare_dss(B, opts->precision, changed)) {
        return rc;
    }
    DevProb v = make_view(P);
    v.r = const_cast<double*>(r);  // read only
    v.z = z;
    v.st = nullptr;
    HIP_TRY(upload_async(B.hook.p, &v, sizeof(v), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const IterArgs ia = iter_args(*opts, -1);
    const DevProb* tab = B.hook.p;
    double* outs[3] = {local_ms, coarse_ms, glue_ms};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int rc = DDMGNN_OK;
    for (int stage = 0; stage < 3 && rc == DDMGNN_OK; ++stage) {
        if (stage == 1 && !opts->coarse) {
            if (outs[1]) *outs[1] = 0.0;
            continue;
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        hipError_t he = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed);
        if (he == hipSuccess) {
            ctx->launch = ctx->cap;
            for (int i = 0; i < reps && rc == DDMGNN_OK && he == hipSuccess; ++i) {
                if (stage == 0)
                    rc = enqueue_dss(B, tab, opts->precision, 1, true, opts->local_solver);
                else if (stage == 1)
                    he = launch_coarse(tab, B.coarse_rows.p, B.n_coarse, ctx->cap, false);
                else
                    he = launch_prolong(tab, B.vec_blk.p, B.n_vec, 1, ia, ctx->cap, false);
            }
            ctx->launch = ctx->stream;
            const hipError_t ee = hipStreamEndCapture(ctx->cap, &g);
            if (he == hipSuccess) he = ee;
        }
        if (he == hipSuccess && rc == DDMGNN_OK) he = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        float ms = 0.f;
        if (he == hipSuccess && rc == DDMGNN_OK) {
            he = hipGraphLaunch(ge, ctx->stream);  // warm-up
            if (he == hipSuccess) he = hipEventRecord(e0, ctx->stream);
            if (he == hipSuccess) he = hipGraphLaunch(ge, ctx->stream);
            if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        }
        if (ge) (void)hipGraphExecDestroy(ge);
        if (he != hipSuccess && rc == DDMGNN_OK) rc = fail(DDMGNN_E_HIP, hipGetErrorString(he));
        if (rc == DDMGNN_OK && outs[stage]) *outs[stage] = (double)ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int ddmgnn_precond_apply(ddmgnn_ctx* ctx, ddmgnn_problem* P, const ddmgnn_solve_opts* opts, const double* r,
                         double* z) {
    if (!ctx || !P || !opts || !r || !z) return fail(DDMGNN_E_INVALID, "null argument");
    if (r == z) return fail(DDMGNN_E_INVALID, "r and z must not alias");
    if (int rc = check_opts(*opts)) return rc;
    if (int rc = solo_batch(P)) return rc;
    Batch& B = *P->solo;
    bool changed = false;
    if (opts->local_solver == DDMGNN_LOCAL_LU) {
        if (int rc = prepare_lu(P)) return rc;
    } else if (int rc = prepare_dss(B, opts->precision, changed)) {
        return rc;
    }
    DevProb v = make_view(P);
    v.r = const_cast<double*>(r);  // read only: the apply never writes its input
    v.z = z;
    v.st = nullptr;
    HIP_TRY(upload_async(B.hook.p, &v, sizeof(v), ctx->stream));
    if (int rc = enqueue_apply(B, B.hook.p, *opts, -1, nullptr, false)) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DDMGNN_OK;
}

int ddmgnn_apply_intermediates(ddmgnn_ctx* ctx, ddmgnn_problem* P, double* s, double* y0, double* y,
                               double* local) {
    if (!ctx || !P) return fail(DDMGNN_E_INVALID, "null argument");
    hipStream_t st = ctx->stream;
    const int K = P->hs.K;
    if (s) HIP_TRY(hipMemcpyAsync(s, P->s.p, K * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (y0) HIP_TRY(hipMemcpyAsync(y0, P->y0.p, K * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (y) HIP_TRY(hipMemcpyAsync(y, P->y.p, K * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (local) HIP_TRY(hipMemcpyAsync(local, P->local.p, P->hs.sk * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return DDMGNN_OK;
}

int ddmgnn_solve(ddmgnn_ctx* ctx, ddmgnn_problem* P, const ddmgnn_solve_opts* opts, double* u_out,
                 ddmgnn_stats* stats) {
    if (!ctx || !P || !opts || !u_out) return fail(DDMGNN_E_INVALID, "null argument");
    if (int rc = check_opts(*opts)) return rc;
    if (int rc = solo_batch(P)) return rc;
    double* outs[1] = {u_out};
    return solve_batch(ctx, *P->solo, *opts, outs, stats);
}

int ddmgnn_solve_batch(ddmgnn_ctx* ctx, ddmgnn_problem* const* probs, int32_t n, const ddmgnn_solve_opts* opts,
                       double* const* u_out, ddmgnn_stats* stats) {
    if (!ctx || !probs || n < 1 || !opts || !u_out) return fail(DDMGNN_E_INVALID, "null argument or n < 1");
    if (int rc = check_opts(*opts)) return rc;
    for (int i = 0; i < n; ++i) {
        if (!probs[i] || !u_out[i]) return fail(DDMGNN_E_INVALID, "null problem or output");
        if (probs[i]->ctx != ctx) return fail(DDMGNN_E_INVALID, "problem belongs to another context");
        if (probs[i]->model->id != probs[0]->model->id)
            return fail(DDMGNN_E_INVALID, "all problems of a batch must share the model");
        for (int j = 0; j < i; ++j)
            if (probs[j] == probs[i]) return fail(DDMGNN_E_INVALID, "a problem appears twice in the batch");
    }
    if (n == 1) return ddmgnn_solve(ctx, probs[0], opts, u_out[0], stats);
    bool hit = ctx->last_batch && (int)ctx->last_batch->ids.size() == n;
    for (int i = 0; hit && i < n; ++i) hit = ctx->last_batch->ids[i] == probs[i]->id;
    if (!hit) {
        ctx->last_batch.reset();
        if (int rc = build_batch(ctx, probs, n, ctx->last_batch)) return rc;
    }
    return solve_batch(ctx, *ctx->last_batch, *opts, u_out, stats);
}

int ddmgnn_expand_overlap(int64_t n_nodes, int64_t n_tri, const int32_t* tri, const int32_t* part, int32_t n_part,
                          int32_t delta, int64_t** sub_ptr_out, int32_t** sub_nodes_out) {
    if (n_nodes <= 0 || n_tri <= 0 || !tri || !part || n_part <= 0 || delta < 0 || !sub_ptr_out || !sub_nodes_out)
        return fail(DDMGNN_E_INVALID, "invalid argument");
    for (int64_t t = 0; t < 3 * n_tri; ++t)
        if (tri[t] < 0 || tri[t] >= n_nodes) return fail(DDMGNN_E_INVALID, "triangle node id out of range");
    for (int64_t i = 0; i < n_nodes; ++i)
        if (part[i] < 0 || part[i] >= n_part) return fail(DDMGNN_E_INVALID, "part id out of range");
    std::vector<int64_t> sp;
    std::vector<int32_t> sn;
    expand_overlap(n_nodes, n_tri, tri, part, n_part, delta, sp, sn);
    auto* a = (int64_t*)std::malloc(sp.size() * sizeof(int64_t));
    auto* b = (int32_t*)std::malloc(std::max<size_t>(1, sn.size()) * sizeof(int32_t));
    if (!a || !b) {
        std::free(a);
        std::free(b);
        return fail(DDMGNN_E_NOMEM, "host allocation failed");
    }
    std::memcpy(a, sp.data(), sp.size() * sizeof(int64_t));
    std::memcpy(b, sn.data(), sn.size() * sizeof(int32_t));
    *sub_ptr_out = a;
    *sub_nodes_out = b;
    return DDMGNN_OK;
}

int ddmgnn_pou_weights(int64_t n_nodes, const uint8_t* dirichlet, int32_t n_sub, const int64_t* sub_ptr,
                       const int32_t* sub_nodes, double* weights_out) {
    if (n_nodes <= 0 || !dirichlet || n_sub <= 0 || !sub_ptr || !sub_nodes || !weights_out)
        return fail(DDMGNN_E_INVALID, "invalid argument");
    std::vector<int32_t> mult(n_nodes, 0);
    for (int64_t k = 0; k < sub_ptr[n_sub]; ++k) {
        if (sub_nodes[k] < 0 || sub_nodes[k] >= n_nodes) return fail(DDMGNN_E_INVALID, "node id out of range");
        mult[sub_nodes[k]]++;
    }
    for (int64_t k = 0; k < sub_ptr[n_sub]; ++k) {
        const int32_t v = sub_nodes[k];
        weights_out[k] = dirichlet[v] ? 0.0 : 1.0 / (double)mult[v];
    }
    return DDMGNN_OK;
}

int ddmgnn_expand_overlap_device(ddmgnn_ctx* ctx, int64_t n_nodes, int64_t n_tri, const int32_t* tri,
                                 const int32_t* part, const uint8_t* dirichlet, int32_t n_part, int32_t delta,
                                 int64_t* sub_ptr_out, int32_t* sub_nodes_out, double* weights_out, int64_t cap) {
    if (!ctx || n_nodes <= 0 || n_nodes > INT32_MAX || n_tri <= 0 || n_tri > INT32_MAX / 3 || !tri || !part ||
        !dirichlet || n_part <= 0 || delta < 0 || !sub_ptr_out || cap < 0 || (cap > 0 && (!sub_nodes_out || !weights_out)))
        return fail(DDMGNN_E_INVALID, "invalid argument");
    hipStream_t s = ctx->stream;
    const int64_t n = n_nodes;
    DevBuf<int> status;
    DevBuf<int32_t> tri_cnt, tri_list, sets0, sets1, part_cnt;
    DevBuf<int64_t> tri_ptr, sub_ptr;
    DevBuf<uint8_t> sz0, sz1;
    HIP_TRY(status.alloc(1));
    HIP_TRY(hipMemsetAsync(status.p, 0, sizeof(int), s));
    HIP_TRY(ov_check(tri, n_tri, part, n, n_part, status.p, s));
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad & 1) return fail(DDMGNN_E_INVALID, "triangle node id out of range");
    if (bad & 2) return fail(DDMGNN_E_INVALID, "part id out of range");
    HIP_TRY(tri_cnt.alloc((size_t)n));
    HIP_TRY(tri_ptr.alloc((size_t)n + 1));
    HIP_TRY(tri_list.alloc((size_t)(3 * n_tri)));
    HIP_TRY(sets0.alloc((size_t)n * OV_CAP));
    HIP_TRY(sets1.alloc((size_t)n * OV_CAP));
    HIP_TRY(sz0.alloc((size_t)n));
    HIP_TRY(sz1.alloc((size_t)n));
    HIP_TRY(part_cnt.alloc((size_t)n_part));
    HIP_TRY(sub_ptr.alloc((size_t)n_part + 1));
    HIP_TRY(hipMemsetAsync(tri_cnt.p, 0, (size_t)n * sizeof(int32_t), s));
    int32_t* sets = nullptr;
    uint8_t* sz = nullptr;
    HIP_TRY(ov_grow(tri, n_tri, part, n, delta, tri_cnt.p, tri_ptr.p, tri_list.p, sets0.p, sets1.p, sz0.p, sz1.p,
                    &sets, &sz, status.p, s));
    HIP_TRY(hipMemsetAsync(part_cnt.p, 0, (size_t)n_part * sizeof(int32_t), s));
    HIP_TRY(ov_count(sets, sz, n, n_part, part_cnt.p, sub_ptr.p, s));
    HIP_TRY(hipMemcpyAsync(sub_ptr_out, sub_ptr.p, ((size_t)n_part + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&bad, status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad & 4) return fail(DDMGNN_E_INVALID, "a node belongs to more than 16 overlapping sub-meshes");
    int64_t kmax = 0;
    for (int32_t i = 0; i < n_part; ++i) kmax = std::max(kmax, sub_ptr_out[i + 1] - sub_ptr_out[i]);
    if (kmax > OV_SORT_MAX) return fail(DDMGNN_E_INVALID, "sub-mesh larger than the supported maximum (16384 nodes)");
    const int64_t sk = sub_ptr_out[n_part];
    if (sk > cap)
        return fail(DDMGNN_E_INVALID, "capacity below sub_ptr_out[n_part] (the number of sub-mesh slots); "
                                      "call again with cap >= sub_ptr_out[n_part]");
    HIP_TRY(hipMemsetAsync(part_cnt.p, 0, (size_t)n_part * sizeof(int32_t), s));
    HIP_TRY(ov_fill(sets, sz, n, dirichlet, n_part, sub_ptr.p, sk, part_cnt.p, sub_nodes_out, weights_out, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DDMGNN_OK;
}

void ddmgnn_free(void* p) { std::free(p); }

}  // extern "C"

int ddmgnn_train_rhs(ddmgnn_ctx* ctx, ddmgnn_problem* P, const double* u, float* c_out) {
    if (!ctx || !P || !u || !c_out) return fail(DDMGNN_E_INVALID, "null argument");
    hipStream_t s = ctx->stream;
    if (P->tr_r.n < (size_t)P->hs.n) HIP_TRY(P->tr_r.alloc((size_t)P->hs.n));
    HIP_TRY(launch_train_rhs(P->rowptr.p, P->col.p, P->val.p, P->b.p, u, P->tr_r.p, (int)P->hs.n, P->sub_ptr.p,
                             P->sub_nodes.p, P->hs.K, c_out, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DDMGNN_OK;
}

int ddmgnn_train_grad(ddmgnn_ctx* ctx, ddmgnn_problem* P, const ddmgnn_model_desc* md, const float* theta,
                      const int32_t* subs, int32_t n, const float* c, const int64_t* c_off, double scale,
                      float* grad, double* loss_out, double* gnorm_out) {
    if (!ctx || !P || !md || !theta || !subs || !c || !c_off || !grad) return fail(DDMGNN_E_INVALID, "null argument");
    if (md->d != D) return fail(DDMGNN_E_INVALID, "training supports the latent width d = 10 only");
    if (md->kbar < 1 || md->kbar > 64) return fail(DDMGNN_E_INVALID, "kbar must be in 1..64");
    if (n < 1) return fail(DDMGNN_E_INVALID, "at least one sample required");
    if (!(scale >= 0.0) || !std::isfinite(scale)) return fail(DDMGNN_E_INVALID, "scale must be finite and >= 0");
    // scratch offsets restart with every chunk of TRAIN_CHUNK samples (one launch each)
    std::vector<int64_t> soff((size_t)n);
    int64_t total = 0, used = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (subs[i] < 0 || subs[i] >= P->hs.K) return fail(DDMGNN_E_INVALID, "sub-mesh index out of range");
        if (P->hs.sub_ptr[subs[i] + 1] - P->hs.sub_ptr[subs[i]] > kMaxSubNodes)
            return fail(DDMGNN_E_INVALID, "training samples are limited to sub-meshes of at most 2048 nodes");
        if (c_off[i] < 0) return fail(DDMGNN_E_INVALID, "negative right-hand side offset");
        if (i % TRAIN_CHUNK == 0) used = 0;
        soff[(size_t)i] = used;
        used += train_scratch_floats(md->kbar, P->hs.sub_ptr[subs[i] + 1] - P->hs.sub_ptr[subs[i]]);
        total = std::max(total, used);
    }
    if (int rc = prepare_train(P)) return rc;
    hipStream_t s = ctx->stream;
    const int64_t nth = (int64_t)md->kbar * TRAIN_NWB;
    if (P->tr_scratch.n < (size_t)total) HIP_TRY(P->tr_scratch.alloc((size_t)total));
    if (P->tr_gpart.n < (size_t)(n * nth)) HIP_TRY(P->tr_gpart.alloc((size_t)(n * nth)));
    if (P->tr_subs.n < (size_t)n) {
        HIP_TRY(P->tr_subs.alloc((size_t)n));
        HIP_TRY(P->tr_coff.alloc((size_t)n));
        HIP_TRY(P->tr_soff.alloc((size_t)n));
        HIP_TRY(P->tr_sse.alloc((size_t)n));
    }
    if (!P->tr_out.p) HIP_TRY(P->tr_out.alloc(2));
    HIP_TRY(upload_async(P->tr_subs.p, subs, (size_t)n * 4, s));
    HIP_TRY(upload_async(P->tr_coff.p, c_off, (size_t)n * 8, s));
    HIP_TRY(upload_async(P->tr_soff.p, soff.data(), (size_t)n * 8, s));
    TrainArgs a{P->sub_ptr.p, P->edge_ptr.p, P->edge_src.p, P->edge_nd.p, P->xy64.p, P->lm_ptr.p, P->lm_col.p,
                P->lm_val.p, P->oe_ptr.p, P->oe_edge.p, P->oe_recv.p, P->tr_subs.p, P->tr_coff.p, P->tr_soff.p,
                c, theta, P->tr_scratch.p, P->tr_gpart.p, P->tr_sse.p, md->kbar, (float)md->alpha, 0};
    for (int32_t s0 = 0; s0 < n; s0 += TRAIN_CHUNK) {
        a.s0 = s0;
        HIP_TRY(launch_train_grad(a, std::min(TRAIN_CHUNK, n - s0), s));
    }
    HIP_TRY(launch_train_reduce(P->tr_gpart.p, n, nth, scale, grad, P->tr_out.p, P->tr_sse.p, s));
    double out2[2];
    HIP_TRY(hipMemcpyAsync(out2, P->tr_out.p, sizeof(out2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss_out) *loss_out = scale * out2[1];
    if (gnorm_out) *gnorm_out = std::sqrt(out2[0]);
    if (!std::isfinite(out2[0]) || !std::isfinite(out2[1]))
        return fail(DDMGNN_E_NONFINITE, "training loss or gradient is not finite");
    return DDMGNN_OK;
}

int ddmgnn_adam_step(ddmgnn_ctx* ctx, float* theta, const float* grad, float* m, float* v, int64_t n, double gnorm,
                     int32_t t, double lr, double beta1, double beta2, double eps, double clip) {
    if (!ctx || !theta || !grad || !m || !v) return fail(DDMGNN_E_INVALID, "null argument");
    if (n < 1 || t < 1) return fail(DDMGNN_E_INVALID, "n >= 1 and step t >= 1 required");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0 && lr >= 0.0))
        return fail(DDMGNN_E_INVALID, "0 <= beta < 1, eps > 0 and lr >= 0 required");
    if (!std::isfinite(gnorm) || gnorm < 0.0) return fail(DDMGNN_E_NONFINITE, "gradient norm is not finite");
    const double gs = clip > 0.0 && gnorm > clip ? clip / gnorm : 1.0;
    const double bc1 = 1.0 - std::pow(beta1, t), bc2 = 1.0 - std::pow(beta2, t);
    HIP_TRY(launch_adam(theta, grad, m, v, n, (float)gs, (float)lr, (float)beta1, (float)beta2, (float)bc1,
                        (float)bc2, (float)eps, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DDMGNN_OK;
}
