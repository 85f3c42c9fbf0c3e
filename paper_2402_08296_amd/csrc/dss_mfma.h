// DSS_theta forward with the MLP layers on BF16 MFMA (v_mfma_f32_32x32x16_bf16).
// Internal interface between the ABI translation unit and dss_mfma.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ddmgnn {

constexpr int MFMA_BLOCK = 1024;  // 16 wavefronts, one sub-mesh per workgroup
constexpr int MFMA_TILE = 32;    // nodes per MFMA tile (the N dimension)

// Per step, per lane of a wavefront: the A operands (8 bf16 per lane, stored
// as raw bits) of the six 32x16 weight tiles, and the lane's FP32 constants.
struct MfmaLane {
    uint16_t aq[8];   // neighbour projections Q' (both message directions)
    uint16_t ap[8];   // receiver projections P'
    uint16_t ah[8];   // Psi hidden layer from (h, 1, c, deg)
    uint16_t asa[8];  // Psi hidden layer from the message sums, units 0..7
    uint16_t asb[8];  // Psi hidden layer from the message sums, units 8..9
    uint16_t a2[8];   // Psi output layer
    float wn[10];     // |d| coefficient of the lane's 10 message units
    float b2[5];      // Psi output bias of the lane's 5 latent components
    float pad;
};
static_assert(sizeof(MfmaLane) == 160, "lane blob layout");

struct MfmaDec {
    uint16_t ad1[8];  // decoder hidden layer from (h, 1)
    uint16_t ad2[8];  // decoder output layer
    float bd2;
    float pad[3];
};
static_assert(sizeof(MfmaDec) == 48, "decoder blob layout");

// Builds the per-lane blobs from the flat FP32 weights (layout of ddmgnn.h).
// The message second layers are folded into the Psi hidden layer
// (no activation lies between them), and the coordinate terms of the message
// first layers are split into receiver and sender parts.
void build_mfma_blobs(const float* theta, int kbar, std::vector<MfmaLane>& lanes, std::vector<MfmaDec>& dec);

struct DssMfmaArgs {
    const int32_t* sub_ptr;
    const int32_t* work_order;
    const int32_t* edge_ptr;     // per slot, in-edge range (global edge index)
    const uint16_t* edge_src;    // per edge, sender local index (padded by 8 entries)
    const float* edge_nd;        // per edge, |d_jl| (padded by 8 entries)
    const uint16_t* tnode;       // per slot position, local node id in tile order (by in-degree)
    const uint16_t* xyhl;        // per slot, bf16 bits of (x_hi, x_lo, y_hi, y_lo), centred coordinates
    const int32_t* sub_nodes;
    const double* weights;
    const double* r;             // apply: global residual
    const double* c_in;          // forward hook: per-slot inputs
    double* out;
    double* s_out;
    double* y0_out;
    float* qglobal;              // Q' storage when it does not fit LDS (20 floats per slot)
    const int* done;             // Krylov converged flag (may be null)
    const MfmaLane* lanes;
    const MfmaDec* dec;
    int kbar;
    float alpha;
    int apply;
    int q_in_lds;
};

// LDS bytes needed for a sub-mesh of k nodes with Q' in LDS.
inline size_t mfma_lds_bytes(int k) { return (size_t)k * (20 + 1) * sizeof(float); }

hipError_t launch_dss_mfma(const DssMfmaArgs& a, int n_sub, size_t shmem, hipStream_t stream);

}  // namespace ddmgnn
