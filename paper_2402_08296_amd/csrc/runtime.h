// Host runtime shared by the C ABI (runtime.cpp) and the serving loop
// (server.cpp): handle layouts, device buffers, batches of problems and the
// solve driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "ddmgnn.h"
#include "device.h"
#include "dss_mfma.h"
#include "setup.h"

namespace ddmgnn {

// Records the error text of the calling thread and returns code.
int fail(int code, const std::string& msg);

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return ::ddmgnn::fail(DDMGNN_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count) {
        reset();
        n = count;
        if (count == 0) return hipSuccess;
        return hipMalloc(&p, count * sizeof(T));
    }
    // Synchronous upload on stream s (the source may be pageable).
    hipError_t upload(const T* src, size_t count, hipStream_t s) {
        hipError_t e = alloc(count);
        if (e != hipSuccess || count == 0) return e;
        e = hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }
};

// Device copy of a model's weights, shared by the model handle and every
// problem created with it (freed with the last of them).
struct ModelDev {
    uint64_t id = 0;
    int kbar = 0;
    int d = D;  // latent width
    bool mfma = true;  // blobs of the matrix-core kernel built (d <= 10: smaller widths zero-padded to 10)
    double alpha = 0;
    DevBuf<float> theta32;
    DevBuf<double> theta64;
    DevBuf<MfmaStep> steps;
    DevBuf<MfmaDec> dec;
};

struct Batch;
struct BatchDeleter {
    void operator()(Batch* b) const;
};
using BatchPtr = std::unique_ptr<Batch, BatchDeleter>;

// Bytes of device memory a problem of these sizes holds (all buffers of a
// solve, excluding the DSS fallback storage of sub-meshes too large for LDS).
size_t problem_device_bytes(int64_t n, int64_t nnz, int32_t K, int64_t sk, int64_t n_edges);

// Creates a problem from a validated descriptor and its host setup (moved in).
// Fills the device-ready host arrays of hs (plain host work; "" or an error).
std::string prepare_upload(const ddmgnn_problem_desc& desc, HostSetup& hs);
// A problem on the device. The copies and the coarse-level kernels run on
// `stream` (the context's stream when null); a server creates problems on a
// stream of its own while the active problems iterate on the context's.
int create_problem(ddmgnn_ctx* ctx, const ddmgnn_problem_desc& desc, std::shared_ptr<ModelDev> model,
                   HostSetup&& hs, ddmgnn_problem** out, hipStream_t stream = nullptr);

// Device buffers of one batched Gauss-Jordan inversion (the plan's arrays,
// scratch and status word).
struct GjBufs {
    DevBuf<int32_t> order, cprefix, tprefix;
    DevBuf<int64_t> prow;
    DevBuf<double> scratch;
    DevBuf<int> status;
};

// Batch of problems solved in lockstep (one launch per kernel and iteration).
// All must share the model. Built once per membership; cheap to rebuild.
int build_batch(ddmgnn_ctx* ctx, ddmgnn_problem* const* probs, int n, BatchPtr& out);

// Prepares the DSS launches for o, uploads the table (with each problem's
// rtol and max_it) and initialises the problems flagged in `init` (none when null).
int batch_begin(Batch& B, const ddmgnn_solve_opts& o, const std::vector<uint8_t>* init);
// Enqueues `count` iterations eagerly (or replays the captured chunk when use_graph).
int batch_iterate(Batch& B, const ddmgnn_solve_opts& o, int count, bool use_graph);
// Copies the states of all problems to the host (synchronises the stream).
int batch_poll(Batch& B);
const KState& batch_state(const Batch& B, int i);
int batch_size(const Batch& B);
ddmgnn_problem* batch_problem(const Batch& B, int i);
// True residuals of the problems flagged in `which` (all when null) into their states, synchronised.
int batch_true_residual(Batch& B, const std::vector<uint8_t>* which);
// Kernel that runs the local solves of problem P: 0 FP64 VALU DSS, 1 FP32 VALU DSS,
// 2 BF16 MFMA DSS, 3 exact local solves (DDM-LU).
// Host copies of a descriptor's arrays when they are device memory.
struct HostDesc {
    std::vector<double> xy, a_val, b, u0, weights;
    std::vector<int32_t> tri, a_rowptr, a_col, sub_nodes;
    std::vector<uint8_t> dirichlet;
    std::vector<int64_t> sub_ptr;
    ddmgnn_problem_desc desc{};
};
// *out = in when its arrays are host memory; else copies them into h (sizes
// from n_nodes, n_tri, n_sub, a_rowptr[N] and sub_ptr[K]) and *out = &h.desc.
int host_desc(const ddmgnn_problem_desc* in, HostDesc& h, const ddmgnn_problem_desc** out);
// Workgroups of a problem in the vector kernels (its tuning, else vec_blocks(n)).
int problem_vec_blocks(const ddmgnn_problem* P);
// Device bytes of the FGMRES storage of a problem of n nodes, cycles of R steps.
size_t fgmres_bytes(int64_t n, int R);
int dss_kernel_of(const ddmgnn_problem* P, const ddmgnn_solve_opts& o);

int check_opts(const ddmgnn_solve_opts& o);

}  // namespace ddmgnn

struct ddmgnn_ctx {
    hipStream_t stream = nullptr;   // the caller's stream: all work runs here
    hipStream_t launch = nullptr;   // where kernels are enqueued (= stream, or cap while capturing)
    hipStream_t cap = nullptr;      // own non-blocking stream for graph capture (the null stream cannot be captured)
    hipStream_t side = nullptr;     // second stream of a forked launch (joined back before the next step)
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    int device = 0;
    ddmgnn::DevBuf<double> partials;
    ddmgnn::DevBuf<double> scalar;
    double* host_pinned = nullptr;
    ddmgnn::BatchPtr last_batch;  // batch of the last multi-problem solve
    ~ddmgnn_ctx();
};

struct ddmgnn_model {
    int kbar = 0, d = 0;
    double alpha = 0;
    std::vector<float> theta;
    std::shared_ptr<ddmgnn::ModelDev> dev;
};

struct ddmgnn_problem {
    ddmgnn_ctx* ctx = nullptr;
    uint64_t id = 0;                 // unique per process (batch cache key)
    ddmgnn::HostSetup hs;
    std::shared_ptr<ddmgnn::ModelDev> model;
    size_t device_bytes = 0;
    // matrix and vectors
    ddmgnn::DevBuf<int32_t> rowptr, col;
    ddmgnn::DevBuf<double> val, b, u0;
    ddmgnn::DevBuf<uint8_t> dirichlet;
    // decomposition
    ddmgnn::DevBuf<int32_t> sub_ptr, sub_nodes, edge_ptr, node_ptr, node_slots, slot_sub;
    // temporaries of the device coarse setup, kept with the problem: freeing them
    // at creation would wait for the work of every stream on the device
    ddmgnn::GjBufs coarse_gj;
    ddmgnn::DevBuf<double> coarse_diag0;
    ddmgnn::DevBuf<int64_t> coarse_off;
    ddmgnn::DevBuf<uint16_t> edge_src;
    ddmgnn::DevBuf<double> weights, xy64, a0inv;
    ddmgnn::DevBuf<float> xyc32;     // per slot, centred on the sub-mesh
    ddmgnn::DevBuf<ddmgnn::TileNode> tiles;
    ddmgnn::DevBuf<uint32_t> erec;   // MFMA kernel edge records, padded per node
    ddmgnn::DevBuf<int32_t> epad_sub;  // [K + 1] ranges of the sub-meshes in erec
    ddmgnn::DevBuf<float> edge_nd;   // padded by 8 entries
    std::vector<uint32_t> mfma_need; // per sub-mesh, LDS bytes of the MFMA kernel (UINT32_MAX: beyond
                                     // its node budget, no tile records)
    std::vector<uint32_t> mfma_need_db;  // the same with two Q' buffers (one barrier per block)
    bool has_big = false;            // a sub-mesh of more than kMaxSubNodes nodes
    ddmgnn_tuning tune{};            // launch schedule (ddmgnn_problem_set_tuning / ddmgnn_autotune)
    // one-sub-mesh forward entry: per-slot input and output, and its one-item work list
    ddmgnn::DevBuf<double> fwd_in, fwd_out;
    ddmgnn::DevBuf<int2> one_work;
    // apply buffers
    ddmgnn::DevBuf<double> s, y0, y, local;
    ddmgnn::DevBuf<double> qglobal64, hglobal64;
    ddmgnn::DevBuf<float> hglobal32;  // FP32 h of the sub-meshes beyond kMaxSubNodes
    ddmgnn::DevBuf<double> cglobal;   // their c (FP64, or FP32 in the same storage)
    // exact local solves (built on the first solve with local_solver = LU)
    ddmgnn::DevBuf<double> lu_inv;
    ddmgnn::DevBuf<int64_t> lu_off;
    // FGMRES basis, preconditioned vectors, partial sums and small arrays (built on
    // the first FGMRES solve, for cycles of up to gm_R steps)
    ddmgnn::DevBuf<double> gm_v, gm_z, gm_part, gm_small;
    int gm_R = 0;
    ddmgnn::DevBuf<float> qglobal32;
    // training: local matrices A_i and out-edge lists (built on the first training
    // call), per-call scratch, per-sample arrays and the residual of ddmgnn_train_rhs
    ddmgnn::DevBuf<int32_t> lm_ptr, oe_ptr, oe_edge, tr_subs;
    ddmgnn::DevBuf<uint16_t> lm_col, oe_recv;
    ddmgnn::DevBuf<float> lm_val, tr_scratch, tr_gpart;
    ddmgnn::DevBuf<int64_t> tr_coff, tr_soff;
    ddmgnn::DevBuf<double> tr_sse, tr_out, tr_r;
    // Krylov vectors
    ddmgnn::DevBuf<double> u, r, z;
    ddmgnn::DevBuf<double> ring;     // (MAX_M + 1) p vectors then (MAX_M + 1) q vectors
    ddmgnn::DevBuf<ddmgnn::KState> st;
    ddmgnn::DevBuf<double> partials;
    double rtol = 1e-6;              // of the current solve (read by the init kernel)
    int max_it = 0;
    ddmgnn::BatchPtr solo;  // batch of this problem alone
    ~ddmgnn_problem();
};
