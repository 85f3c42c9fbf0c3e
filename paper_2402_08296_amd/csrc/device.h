// Device-side types shared by the kernel translation units and the host
// runtime: Krylov scalars, the per-problem pointer table, work items and the
// kernel launchers.
//
// Every kernel is table driven. A launch serves one or several problems (a
// batch): workgroup b looks up its work item (problem index, sub-mesh / row /
// local workgroup) and reads that problem's pointers from the table. A single
// solve is a batch of one. Problems that have converged keep their slots in
// the grid but their workgroups return at once (the per-problem done flag).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ddmgnn {

constexpr int D = 10;           // latent width of the paper's model (Sec. IV.B); the MFMA kernel's width
constexpr int MAX_M = 4;        // largest FCG truncation supported
constexpr int MAX_RESTART = 64; // largest FGMRES cycle
constexpr int VEC_BLOCK = 256;  // threads of the vector kernels
constexpr int VEC_GRID = 1024;  // max workgroups per problem in the vector kernels
constexpr int N_XCD = 8;        // accelerator dies; workgroups are dispatched to them round-robin
constexpr int DSS_BLOCK = 512;  // threads of the VALU DSS kernel
constexpr int DSS_WIDE_BLOCK = 1024;  // its form for launches of fewer sub-meshes than compute units
constexpr int N_CU = 256;  // compute units of an MI355X
constexpr size_t LDS_LIMIT = 160 * 1024;

// Krylov scalars of one problem, resident in device memory.
struct KState {
    double r0n;            // |r_0|
    double rtol;
    double rel;            // |r_it| / |r_0|
    double alpha;
    double beta[MAX_M];    // p_new = z + sum_k beta[k] p_(it-1-k)
    double pq[MAX_M + 1];  // <p, A p> of each direction-ring slot
    double rho;            // PCG/CG: <r, z> of the current iteration
    double rr_true;        // |b - A u|^2 at exit
    int it;                // completed iterations
    int done;
    int status;
    int max_it;            // the update kernel raises done once it reaches max_it
    // FGMRES cycle (unused by the other methods)
    double gm_beta;        // |r| at the start of the cycle
    double gm_hnext;       // h_{j,j-1}: norm of the unnormalised basis vector j
    int gm_j;              // step of the cycle (basis vectors 0..gm_j exist)
    int gm_k;              // steps of a finished cycle
    int gm_end;            // the cycle is over: update u, restart or stop
    int gm_conv;           // the residual estimate met the tolerance
};

// Per slot position in tile order (nodes of a sub-mesh by decreasing
// in-degree): the node's local id, in-degree, first padded in-edge record, and the bf16 bits
// of its sub-mesh-centred coordinates split as x = x_hi + x_lo, y = y_hi + y_lo.
struct TileNode {
    int32_t e0;
    uint16_t j;
    uint16_t deg;
    uint16_t xh, xl, yh, yl;
};
static_assert(sizeof(TileNode) == 16, "tile record layout");

// Device view of one problem (all pointers device memory).
struct DevProb {
    // matrix, right-hand side, boundary
    const int32_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* b;
    const double* u0;
    const uint8_t* dirichlet;
    // decomposition and DSS graphs (slot = position in sub_nodes)
    const int32_t* sub_ptr;
    const int32_t* sub_nodes;
    const double* weights;
    const int32_t* edge_ptr;    // per slot, in-edge range (global edge index)
    const uint16_t* edge_src;   // per edge, sender local id; padded by 8 entries
    const float* edge_nd;       // per edge, |d_jl|; padded by 8 entries
    const uint32_t* erec;       // per node of each sub-mesh, its in-edges (FP16 |d_jl| | 20 * sender << 16)
                                // padded with sentinel records (sender k_i, |d| 0) to a multiple of MFMA_EC
    const int32_t* epad_sub;    // [K + 1] range of each sub-mesh in erec
    const TileNode* tiles;      // per slot position in tile order (e0 indexes erec)
    const double* xy64;         // per slot, raw coordinates
    const float* xyc32;         // per slot, sub-mesh-centred coordinates
    const int32_t* node_ptr;    // per node, range of its slots
    const int32_t* node_slots;
    const int32_t* slot_sub;
    const double* a0inv;        // K x K
    const double* lu_inv;       // local exact solves: (R_i A R_i^T)^{-1} per sub-mesh, k_i rows of
                                // stride k_i rounded up to even (16-byte aligned rows, zero pad)
    const int64_t* lu_off;      // [K + 1] offsets into lu_inv (null until built)
    // iteration vectors
    double* u;
    double* r;                  // residual; input of the apply
    double* z;                  // output of the apply
    const double* c_in;         // DSS forward entry: per-slot inputs (null in solves)
    double* p[MAX_M + 1];       // direction ring
    double* q[MAX_M + 1];       // A p of each ring slot
    double* s;                  // [K] |R_i r|
    double* y0;                 // [K] R_0 r
    double* y;                  // [K] coarse solution
    double* local;              // per slot, |R_i r| r~_i (or r~_i for the forward entry)
    double* qg64;               // DSS fallback storage when LDS is too small (may be null)
    double* hg64;               // FP64 DSS latent state
    float* qg32;
    float* hg32;                // FP32 latent state of sub-meshes beyond the register-resident size
    double* c64;                // normalised local right-hand sides of those sub-meshes (FP64 form),
    float* c32;                 // and the same storage read as FP32 (FP32 form)
    KState* st;                 // null: no Krylov scalars, no done flag
    double* partials;           // (MAX_M + 1) x VEC_GRID per-workgroup partial sums
    // FGMRES storage (null until a problem is solved with FGMRES)
    double* gm_v;               // (restart + 1) x n: Arnoldi basis V
    double* gm_z;               // restart x n: preconditioned vectors Z = M(V)
    double* gm_part;            // (restart + 1) x VEC_GRID partial sums of the Gram passes
    double* gm_small;           // H [(restart + 1) x restart, column j at j * (restart + 1)],
                                // cs, sn [restart], g [restart + 1], y [restart], tmp [restart + 1]
    double rtol;                // read by the init kernel
    int max_it;
    int n;
    int K;
    int nblk;                   // workgroups of this problem in the vector kernels
};

// Options of one Krylov iteration, common to the problems of a launch.
struct IterArgs {
    int mode;        // DDMGNN_FCG / PCG / CG / FGMRES; < 0: bare apply (no Krylov scalars)
    int m;           // directions kept (FCG m_max; 1 for PCG and CG); FGMRES: cycle length
    int unweighted;  // gluing without partition-of-unity weights
    int coarse;      // add the coarse correction
};

// Ring slots of iteration `it` with `m` kept directions: the new direction
// goes to it % (m+1), previous direction k (0 = most recent) is in (it-1-k) mod (m+1).
__host__ __device__ inline int ring_cur(int it, int m) { return it % (m + 1); }
__host__ __device__ inline int ring_prev(int it, int m, int k) {
    const int nr = m + 1;
    return ((it - 1 - k) % nr + nr) % nr;
}

// Launchers (kernels.hip). tab: device table; the int2 lists are device
// arrays of (problem, item) pairs, one per workgroup. check = false skips
// hipGetLastError (not allowed while a stream is being captured).
hipError_t prepare_dss_valu(int precision, int d, size_t shmem);
hipError_t launch_dss_valu(const DevProb* tab, const int2* work, int n_work, int precision, int d, bool qlds,
                           int kbar, double alpha, int apply, const float* theta32, const double* theta64,
                           size_t shmem, hipStream_t s, bool check);
// The VALU DSS forward for sub-meshes of more than kMaxSubNodes nodes (h, c
// and Q in the per-slot global buffers hg32/hg64, c32/c64, qg32/qg64).
hipError_t launch_dss_big(const DevProb* tab, const int2* work, int n_work, int precision, int d, int kbar,
                          double alpha, int apply, const float* theta32, const double* theta64, hipStream_t s,
                          bool check);
// Exact local solves (DDM-LU): restriction as in the DSS kernels, then
// local = (R_i A R_i^T)^{-1} R_i r per sub-mesh; R_i r is staged in dynamic
// LDS of max_k doubles (the largest sub-mesh of the work list).
// prepare_lu_local raises the kernel's LDS limit to kMaxSubNodesAny doubles
// (not allowed during stream capture).
hipError_t prepare_lu_local();
// Device factorisation (factor.hip). launch_lu_assemble: A_i = R_i A R_i^T of
// every sub-mesh, dense, sub-mesh i at off[i] of inv with row stride
// (off[i + 1] - off[i]) / k_i. launch_coarse_assemble: A_0 = R_0 A R_0^T (K x K,
// deterministic summation order), symmetrised, its diagonal copied to diag0.
// launch_gj_invert: in-place inverses of a batch of SPD matrices (matrix m at
// base + off[m], order plan.order[m]) by blocked Gauss-Jordan over the whole
// device; scratch holds plan.scratch_doubles(); *status (device, zeroed by the
// caller) gets bit 0 when a pivot is not positive (or, with diag0, below 1e-12
// of its original diagonal entry).
struct GjPlan {
    std::vector<int32_t> order, cprefix, tprefix;  // orders; workgroup prefixes (columns, tiles)
    std::vector<int64_t> prow;                     // prefix of the orders
    int32_t max_k = 0;
    int64_t tiles = 0;  // tile workgroups of one trailing update
    explicit GjPlan(const std::vector<int32_t>& k);
    size_t scratch_doubles() const;
};
struct GjPlanDev {  // device copies of a plan's arrays
    const int32_t* order;
    const int32_t* cprefix;
    const int32_t* tprefix;
    const int64_t* prow;
};
hipError_t launch_lu_assemble(const int32_t* rowptr, const int32_t* col, const double* val, const int64_t* sub_ptr,
                              const int32_t* sub_nodes, const int64_t* off, double* inv, int n_sub, hipStream_t s);
hipError_t launch_coarse_assemble(const int32_t* rowptr, const int32_t* col, const double* val,
                                  const int32_t* sub_ptr, const int32_t* sub_nodes, const double* weights,
                                  const int32_t* node_ptr, const int32_t* node_slots, const int32_t* slot_sub, int K,
                                  double* a0, double* diag0, hipStream_t s);
hipError_t launch_gj_invert(const GjPlan& plan, const GjPlanDev& dev, double* base, const int64_t* off,
                            double* scratch, const double* diag0, int* status, hipStream_t s);
// Overlap expansion on the device (overlap.hip). OV_CAP: most sub-meshes a node
// may belong to; OV_SORT_MAX: largest sub-mesh the per-part sort holds (the
// library's sub-mesh limit). ov_check: bit 0 of *status for a triangle node id
// out of [0, n), bit 1 for a part id out of [0, n_part). ov_grow: node ->
// triangle lists (tri_cnt must be zero), then delta rounds of growth of the
// per-node part sets (bit 2 of *status on overflow); *sets_out / *sz_out point
// at the final sets. ov_count: sub-mesh sizes (part_cnt zero) and their
// exclusive scan sub_ptr[0..n_part]. ov_fill: the sorted lists and weights
// (part_cur zero).
constexpr int OV_CAP = 16;
constexpr int OV_SORT_MAX = 16384;
hipError_t ov_check(const int32_t* tri, int64_t n_tri, const int32_t* part, int64_t n, int32_t n_part, int* status,
                    hipStream_t s);
hipError_t ov_grow(const int32_t* tri, int64_t n_tri, const int32_t* part, int64_t n, int32_t delta,
                   int32_t* tri_cnt, int64_t* tri_ptr, int32_t* tri_list, int32_t* sets0, int32_t* sets1,
                   uint8_t* sz0, uint8_t* sz1, int32_t** sets_out, uint8_t** sz_out, int* status, hipStream_t s);
hipError_t ov_count(const int32_t* sets, const uint8_t* sz, int64_t n, int32_t n_part, int32_t* part_cnt,
                    int64_t* sub_ptr, hipStream_t s);
hipError_t ov_fill(const int32_t* sets, const uint8_t* sz, int64_t n, const uint8_t* dirichlet, int32_t n_part,
                   const int64_t* sub_ptr, int64_t sk, int32_t* part_cur, int32_t* nodes, double* weights,
                   hipStream_t s);
hipError_t launch_lu_local(const DevProb* tab, const int2* work, int n_work, int max_k, hipStream_t s, bool check);
hipError_t launch_coarse(const DevProb* tab, const int2* rows, int n_rows, hipStream_t s, bool check);
// The Krylov launchers end with a finalize launch of one workgroup per
// problem: n_prob = all problems of the table, or the problems of `list`.
hipError_t launch_prolong(const DevProb* tab, const int2* blk, int n_blk, int n_prob, const IterArgs& it,
                          hipStream_t s, bool check);
// FGMRES: one step of every problem of the table (after its apply) and the
// normalisation that starts the next step (before it).
hipError_t launch_fgmres_next(const DevProb* tab, const int2* blk, int n_blk, const IterArgs& it, hipStream_t s,
                              bool check);
hipError_t launch_fgmres_step(const DevProb* tab, const int2* blk, int n_blk, int n_prob, const IterArgs& it,
                              hipStream_t s, bool check);
hipError_t launch_krylov(const DevProb* tab, const int2* blk, int n_blk, int n_prob, const IterArgs& it,
                         hipStream_t s, bool check);
hipError_t launch_init(const DevProb* tab, const int2* blk, int n_blk, const int* list, int n_list, hipStream_t s);
hipError_t launch_resid(const DevProb* tab, const int2* blk, int n_blk, const int* list, int n_list, hipStream_t s);
hipError_t launch_gather_states(const DevProb* tab, int n, KState* out, hipStream_t s);
// Entry points: y = A x with the solve's grouped SpMV over nblk workgroups, and
// *out = x.y (device) with the solve's two-kernel reduction (partials: VEC_GRID
// doubles of scratch); n < 2^31.
hipError_t launch_spmv(const int32_t* rowptr, const int32_t* col, const double* val, const double* x, double* y,
                       int n, int nblk, hipStream_t s);
hipError_t launch_dot(const double* x, const double* y, int n, double* partials, double* out, hipStream_t s,
                      bool check);

// Allocation-free entry points (noalloc.hip): a static device array of
// NOALLOC_SCRATCH_DOUBLES doubles per device holds their scratch. noalloc_init
// looks up the array's device address on the current device (once per device);
// noalloc_scratch returns it (nullptr before noalloc_init ran on that device).
constexpr int NOALLOC_SCRATCH_DOUBLES = VEC_GRID;  // the dot product's partial sums
hipError_t noalloc_init(int device);
double* noalloc_scratch(int device);

// Training of DSS_theta (train.hip): one TRAIN_BLOCK-thread workgroup per local
// problem; TRAIN_NWB weights per block (d = D).
constexpr int TRAIN_BLOCK = 1024;
constexpr int TRAIN_NWB = 11 * D * D + 15 * D + 1;
struct TrainArgs {
    const int32_t* sub_ptr;
    const int32_t* edge_ptr;   // per slot, in-edge range
    const uint16_t* edge_src;  // per in-edge, sender local id
    const float* edge_nd;      // per in-edge, |d|
    const double* xy64;        // per slot, coordinates
    const int32_t* lm_ptr;     // per slot, range of its row of A_i = R_i A R_i^T
    const uint16_t* lm_col;    // local column
    const float* lm_val;
    const int32_t* oe_ptr;     // per slot, range of its out-edges
    const int32_t* oe_edge;    // the in-edge index of each out-edge
    const uint16_t* oe_recv;   // its receiver's local id
    const int32_t* subs;       // per sample: sub-mesh,
    const int64_t* c_off;      // offset of its right-hand side in c,
    const int64_t* s_off;      // offset of its scratch
    const float* c;
    const float* theta;        // kbar blocks of TRAIN_NWB weights
    float* scratch;
    float* gpart;              // per sample, kbar * TRAIN_NWB weight gradients
    double* sse;               // per sample, sum of squared residuals over the blocks
    int kbar;
    float alpha;
    int s0;                    // first sample of this launch (workgroup b takes sample s0 + b)
};
// Samples per launch of the training kernel: launches reuse one scratch region.
constexpr int TRAIN_CHUNK = 512;
int64_t train_scratch_floats(int kbar, int64_t k);
hipError_t launch_train_grad(const TrainArgs& a, int n, hipStream_t s);
// grad = scale * sum over samples of gpart; out2[0] = |grad|^2, out2[1] = sum of sse.
hipError_t launch_train_reduce(const float* gpart, int n, int64_t nth, double scale, float* grad, double* out2,
                               const double* sse, hipStream_t s);
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int64_t n, float gscale, float lr,
                       float b1, float b2, float bc1, float bc2, float eps, hipStream_t s);
// r = b - A u, then c = R_i r / |R_i r| per sub-mesh (slot order).
hipError_t launch_train_rhs(const int32_t* rowptr, const int32_t* col, const double* val, const double* bb,
                            const double* u, double* r, int n, const int32_t* sub_ptr, const int32_t* sub_nodes,
                            int K, float* c, hipStream_t s);

// Workgroups a problem of n rows takes in the vector kernels.
// Workgroups of a problem in the vector kernels: one per VEC_BLOCK rows up to
// VEC_GRID, rounded up to a multiple of N_XCD (so that a problem's workgroups
// start on die 0 in every launch and split evenly over the dies).
inline int vec_blocks(int64_t n) {
    int64_t g = (n + VEC_BLOCK - 1) / VEC_BLOCK;
    g = g > VEC_GRID ? VEC_GRID : g;
    g = (g + N_XCD - 1) / N_XCD * N_XCD;
    return (int)(g < N_XCD ? N_XCD : g);
}
static_assert(VEC_GRID % N_XCD == 0, "vector grid must split over the dies");

}  // namespace ddmgnn
