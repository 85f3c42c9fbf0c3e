// Host-side setup of a DDM-GNN problem (no device code): validation, overlap
// expansion, local DSS graphs, membership lists and the coarse operator.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ddmgnn.h"

namespace ddmgnn {

constexpr int kMaxSubNodes = 2048;  // largest sub-mesh the DSS kernels accept

// Returns an empty string when desc is valid, else the reason.
std::string validate(const ddmgnn_problem_desc& d);

void expand_overlap(int64_t n, int64_t nt, const int32_t* tri, const int32_t* part, int32_t n_part,
                    int32_t delta, std::vector<int64_t>& sub_ptr, std::vector<int32_t>& sub_nodes);

struct HostSetup {
    int64_t n = 0, nnz = 0, sk = 0, n_edges = 0;
    int32_t K = 0;
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
};

// Local DSS graphs, slot_sub, node membership lists and work order only.
void build_local_graphs(const ddmgnn_problem_desc& d, HostSetup& s);

// Builds everything above. Returns "" on success, "NOT_SPD" if the coarse
// Cholesky fails, else an error message.
std::string build_setup(const ddmgnn_problem_desc& d, HostSetup& s);

}  // namespace ddmgnn
