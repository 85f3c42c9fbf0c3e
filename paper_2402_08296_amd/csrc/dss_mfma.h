// DSS_theta forward with the MLP layers on BF16 MFMA (v_mfma_f32_32x32x16_bf16).
// Internal interface between the ABI translation unit and dss_mfma.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device.h"

namespace ddmgnn {

constexpr int MFMA_BLOCK = 1024;  // 16 wavefronts, one sub-mesh per workgroup
// Sub-meshes of at most MFMA_SMALL_K nodes may run in workgroups of
// MFMA_SMALL_BLOCK threads instead: two fit on a compute unit when each needs at
// most half its LDS, and one's barrier waits are the other's issue slots.
constexpr int MFMA_SMALL_BLOCK = 512;
constexpr int MFMA_SMALL_K = 1024;
constexpr size_t MFMA_SMALL_LDS = 80 * 1024 - 1024;  // largest dynamic LDS of two co-resident workgroups
constexpr int MFMA_TILE = 32;    // nodes per MFMA tile (the N dimension)
// Edges per straight-line chunk of the message sums. Each node's in-edge
// records are padded to a multiple of it with records of a sentinel sender
// whose projections are -inf, so a padded edge contributes ReLU(-inf) = 0.
constexpr int MFMA_EC = 2;

// Edge record of the MFMA kernel: FP16 bits of |d_jl| in the low half, the
// byte offset of the sender's row in a direction's Q' array (5 dwords per
// row) in the high half.
inline uint32_t mfma_edge_record(int sender, uint16_t nd_fp16_bits) {
    return (uint32_t)nd_fp16_bits | ((uint32_t)(sender * 20) << 16);
}

// Per step: the A operands (8 values per lane, raw bits) of the six 32x16
// weight tiles and the lanes' FP32 constants, stored structure-of-arrays
// ([field][lane]) so that the 64 lanes read consecutive addresses. The tiles
// are bf16, except the two that multiply the FP16 message sums (fp16).
enum { A_Q = 0, A_P = 1, A_H = 2, A_SA = 3, A_SB = 4, A_2 = 5, N_ATILES = 6 };
struct MfmaStep {
    uint16_t a[N_ATILES][64][8];  // Q', P', Psi hidden from (h,1,c,deg), from sums 0..7, 8..9, Psi output (with bias)
    uint32_t wn2[5][64];          // |d| coefficients of the lane's 10 message units, FP16 pairs (2t, 2t+1)
};
static_assert(sizeof(MfmaStep) % 16 == 0, "step blob is copied in 16-byte units");

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
void build_mfma_blobs(const float* theta, int kbar, std::vector<MfmaStep>& steps, std::vector<MfmaDec>& dec);
// A model of latent width d < 10 in the layout of width 10: its weights in the
// leading rows and columns of every matrix and vector, zeros elsewhere. The
// padded hidden units and latent components then stay exactly 0 (ReLU(0) = 0,
// zero output rows), so the width-10 network computes the width-d one.
void pad_theta_to_d10(const float* theta, int kbar, int d, std::vector<float>& out);

struct DssMfmaArgs {
    const DevProb* tab;          // per problem: graphs, tile records, vectors, done flag
    const int2* work;            // (problem, sub-mesh) per workgroup, largest sub-meshes first
    const MfmaStep* steps;
    const MfmaDec* dec;
    int kbar;
    float alpha;
    int apply;                   // 1: restrict P.r and write s r~ to P.local; 0: read P.c_in, write r~
    uint32_t lds_bytes;          // dynamic LDS of the launch (set by launch_dss_mfma)
};

// LDS of a workgroup: c (k floats), one or two (db) Q' buffers of
// 2 x (k + 1) x 5 dwords (the last row of each direction the sentinel),
// padded edge records (ne_pad uint32), each region padded to 16 bytes, then
// tile records (k x 16 bytes). A sub-mesh whose single-buffer need exceeds the
// limit is not run by this kernel; one whose double-buffer need fits the
// launch's dynamic LDS runs with two buffers.
constexpr size_t MFMA_LDS_LIMIT = 160 * 1024 - 1024;
__host__ __device__ inline size_t mfma_lds_need(int k, int64_t ne_pad, bool db = false) {
    return (size_t)((k + 3) & ~3) * 4 + (size_t)(db ? 2 : 1) * (size_t)((10 * ((int64_t)k + 1) + 3) & ~3) * 4 +
           (size_t)((ne_pad + 3) & ~3) * 4 + (size_t)k * 16;
}

// Sets the dynamic-LDS limit of the kernel (not allowed during stream capture).
hipError_t prepare_dss_mfma(size_t shmem);
// block: MFMA_BLOCK, or MFMA_SMALL_BLOCK for a list of sub-meshes of at most
// MFMA_SMALL_K nodes. check = false skips hipGetLastError (used while a stream
// is being captured).
hipError_t launch_dss_mfma(const DssMfmaArgs& a, int n_work, size_t shmem, int block, hipStream_t stream,
                           bool check);

}  // namespace ddmgnn
