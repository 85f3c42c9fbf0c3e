// Host-side setup of a DDM-GNN problem (no device code): validation, overlap
// expansion, local DSS graphs, membership lists and the coarse operator.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "ddmgnn.h"

namespace ddmgnn {

// Indices 0..n-1 spread over host threads; each index is handled by one thread,
// so results do not depend on the thread count.
template <class F>
void parallel_for(int64_t n, F&& f) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t T = std::min<int64_t>({n, (int64_t)hw, 16});
    if (T <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next{0};
    auto work = [&] {
        for (int64_t i = next.fetch_add(1); i < n; i = next.fetch_add(1)) f(i);
    };
    std::vector<std::thread> th;
    for (int64_t t = 1; t < T; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
}

constexpr int kMaxSubNodes = 2048;      // largest sub-mesh of the register-resident DSS kernels
constexpr int kMaxSubNodesAny = 16384;  // largest sub-mesh accepted (16-bit local ids; DDM-LU stages
                                        // R_i r in 128 KiB of LDS)

// Returns an empty string when desc is valid, else the reason.
std::string validate(const ddmgnn_problem_desc& d);

void expand_overlap(int64_t n, int64_t nt, const int32_t* tri, const int32_t* part, int32_t n_part,
                    int32_t delta, std::vector<int64_t>& sub_ptr, std::vector<int32_t>& sub_nodes);

struct HostSetup {
    int64_t n = 0, nnz = 0, sk = 0, n_edges = 0;
    int32_t K = 0;
    std::vector<int64_t> sub_ptr;    // [K + 1] slot ranges of the sub-meshes
    // Local DSS graphs, one receiver-major CSR per sub-mesh, concatenated:
    // rows of sub-mesh i are slots sub_ptr[i]..sub_ptr[i+1]; edge_ptr[slot]
    // indexes edge_src (sender slot, local id) for the in-edges of that slot.
    std::vector<int64_t> edge_ptr;   // [sk + 1]
    std::vector<uint16_t> edge_src;  // [n_edges] sender local index
    std::vector<int32_t> slot_sub;   // [sk] sub-mesh of each slot
    // Membership of each node: node_ptr[n]..node_ptr[n+1] index node_slots.
    std::vector<int64_t> node_ptr;   // [n + 1]
    std::vector<int32_t> node_slots; // [sk]
    // Coarse operator A_0 = Z^T A Z (Z = R_0^T) and its inverse, row-major K x K.
    std::vector<double> a0, a0inv;
    // Sub-meshes ordered by decreasing size (largest first) for the DSS launch.
    std::vector<int32_t> work_order;
    int32_t max_k = 0;
    // For the MFMA kernel: per slot position, the local node id in order of
    // decreasing in-degree (tiles of nodes with similar degree); per slot, the
    // bf16 bits of (x_hi, x_lo, y_hi, y_lo) of the coordinates relative to the
    // sub-mesh centroid; per edge, |d_jl| in FP32.
    std::vector<uint16_t> tnode;
    std::vector<uint16_t> xyhl;
    std::vector<double> xyc;   // per slot, coordinates relative to the sub-mesh centroid
    std::vector<uint32_t> erec;  // per edge: sender local id | FP16 bits of |d_jl| << 16
    int64_t max_edges_sub = 0;   // largest in-edge count of a sub-mesh
    std::vector<float> edge_nd;
    // Exact local solves, when built before the problem is created: inverses
    // of R_i A R_i^T, row stride lu_ld(k_i), sub-mesh i at lu_off[i] (empty otherwise).
    std::vector<double> lu_inv;
    std::vector<int64_t> lu_off;
    // Device-ready arrays, filled by prepare_upload (the setup workers of a server
    // run it, so that admission only copies): 32-bit index arrays, the slot
    // coordinates (FP64 raw, FP32 centred), the padded edge arrays, and the records
    // of the matrix-core DSS kernel (per sub-mesh edge-block offsets, slot-major edge
    // records, 16-byte tile records as four words each, and the LDS need with one and
    // two Q' buffers, UINT32_MAX for a sub-mesh that runs the VALU kernel).
    bool upload_ready = false;
    bool has_big = false;
    std::vector<int32_t> sp32, ep32, np32;
    std::vector<double> xy64;
    std::vector<float> xyc32, nd_pad;
    std::vector<uint16_t> src_pad;
    std::vector<uint32_t> mfma_erec, mfma_tiles, mfma_need, mfma_need_db;
    std::vector<int32_t> mfma_epad;
};

// Inverse of the local matrix R_i A R_i^T of sub-mesh i (dense, row-major
// k_i x k_i; the paper's exact local solve of DDM-LU) by Cholesky. "" or "NOT_SPD".
std::string local_inverse(const ddmgnn_problem_desc& d, int32_t i, std::vector<double>& inv, bool parallel);
// Row stride of a stored local inverse: k rounded up to even, so that every row
// starts 16-byte aligned (the pad column holds zeros).
inline int64_t lu_ld(int64_t k) { return (k + 1) & ~int64_t(1); }
// All local inverses concatenated, sub-mesh i at off[i] = sum_{j < i} k_j lu_ld(k_j)
// with row stride lu_ld(k_i) (sub-meshes in parallel).
std::string build_local_inverses(const ddmgnn_problem_desc& d, std::vector<double>& inv, std::vector<int64_t>& off);

// Round-to-nearest-even float -> bf16 bits.
inline uint16_t bf16_rne_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
inline float bf16_bits_float(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Local DSS graphs, slot_sub, node membership lists and work order only.
void build_local_graphs(const ddmgnn_problem_desc& d, HostSetup& s);

// Builds everything above (the coarse operator and its inverse only when
// `coarse`; the library forms them on the device). Returns "" on success,
// "NOT_SPD" if the coarse Cholesky fails, else an error message.
std::string build_setup(const ddmgnn_problem_desc& d, HostSetup& s, bool coarse = true);

}  // namespace ddmgnn
