// DSS_theta forward pass (Sec. III.B, eqs. (14)-(18)) with the dense MLP
// layers on BF16 MFMA and FP32 accumulation.
//
// Layout. A wavefront processes tiles of 32 nodes: the nodes are the N
// dimension of v_mfma_f32_32x32x16_bf16, the features the M and K dimensions.
// Lane l serves node (l % 32) of the tile and half hf = l / 32. An MFMA output
// row r lands in item 4*(r/8) + r%4 of the lanes with hf = (r/4)%2, and a B
// operand lane holds the 8 consecutive K entries 8*hf..8*hf+7, so a layer's
// output items feed the next layer's B operand without moving data between
// lanes once the weight rows and columns are permuted to match (done on the
// host in build_mfma_blobs). Half hf of a node holds:
//   * latent components 5*hf .. 5*hf+4 of h (FP32, registers, all kbar blocks);
//   * message units 0..9 of direction hf (hf = 0: Phi_out, hf = 1: Phi_in).
//
// One block k:
//   Q'_l = W1[:, h_l] h_l + W1[:, d] x_l        (per node, MFMA; stored to LDS in FP16)
//   P'_j = W1[:, h_j] h_j + b1 - W1[:, d] x_j    (per node, MFMA)
//   S_j  = sum_{l in N(j)} ReLU(P'_j + Q'_l + w_|d| |d_jl|)   (per edge, VALU)
// which equals sum_l ReLU(W1 (h_j, h_l, d_jl, |d_jl|) + b1) because d_jl =
// x_l - x_j (for Phi_in the signs of the coordinate terms flip, d_lj = -d_jl).
// Coordinates enter the MFMA as bf16 hi/lo pairs of sub-mesh-centred values,
// so the large per-node terms cancel to FP32 accuracy in P' + Q'. Then
//   hid = ReLU(W1_psi (h, c, phi_out, phi_in) + b1_psi) with phi = W2 S + deg b2
// is one MFMA chain over (h, 1, c, deg) and S (the second message layers are
// folded into W1_psi on the host), and h += alpha (W2_psi hid + b2_psi).
#include "dss_mfma.h"

#include <cmath>
#include <cstring>

namespace ddmgnn {

namespace {

constexpr int IN_PHI = 2 * D + 3;
constexpr int IN_PSI = 3 * D + 1;
constexpr int OFF_PO = 0;
constexpr int OFF_PI = OFF_PO + D * IN_PHI + D + D * D + D;
constexpr int OFF_PS = OFF_PI + D * IN_PHI + D + D * D + D;
constexpr int OFF_DE = OFF_PS + D * IN_PSI + D + D * D + D;
constexpr int BLOCK_W = OFF_DE + D * D + D + D + 1;
constexpr int EC = MFMA_EC;
// Tiles a wavefront holds (h in registers): a 1024-thread workgroup takes any
// sub-mesh (64 tiles at most), a 512-thread one those of up to MFMA_SMALL_K nodes.
constexpr int MAX_TILES_PER_WAVE = 4;
static_assert(MAX_TILES_PER_WAVE * (MFMA_BLOCK / 64) * MFMA_TILE >= 2048, "largest sub-mesh");
static_assert(MAX_TILES_PER_WAVE * (MFMA_SMALL_BLOCK / 64) * MFMA_TILE >= MFMA_SMALL_K, "small sub-meshes");

// Round-to-nearest-even float -> bf16 bits (host).
uint16_t bf16_bits(double v) {
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// K-index roles of the B operands (k = 8*hf + m).
enum Role { H, ONE, XHI, XLO, YHI, YLO, C, DEG, ZERO };
// Both halves carry the same kinds of entries at m = 5..7, so the kernel
// builds its B operands without selecting on the half; an entry whose role is
// ZERO meets a zero weight column.
Role pq_role(int k, int* hidx) {
    const int hf = k / 8, m = k % 8;
    if (m < 5) { *hidx = 5 * hf + m; return H; }
    if (hf == 0) return m == 5 ? XHI : (m == 6 ? XLO : ONE);
    return m == 5 ? YHI : (m == 6 ? YLO : ZERO);
}
Role psi_role(int k, int* hidx) {
    const int hf = k / 8, m = k % 8;
    if (m < 5) { *hidx = 5 * hf + m; return H; }
    if (hf == 0) return m == 5 ? ONE : (m == 6 ? C : DEG);
    return ZERO;
}
// Output row r -> (half, item) of the lanes that receive it.
inline int row_half(int r) { return (r / 4) % 2; }
inline int row_item(int r) { return 4 * (r / 8) + r % 4; }

}  // namespace

void pad_theta_to_d10(const float* theta, int kbar, int d, std::vector<float>& out) {
    const int in_phi = 2 * d + 3, in_psi = 3 * d + 1, bw = 11 * d * d + 15 * d + 1;
    out.assign((size_t)kbar * BLOCK_W, 0.0f);
    for (int step = 0; step < kbar; ++step) {
        const float* src = theta + (size_t)step * bw;
        float* dst = out.data() + (size_t)step * BLOCK_W;
        // message MLPs: inputs (h_j, h_l, d_x, d_y, |d|)
        for (int dir = 0; dir < 2; ++dir) {
            const float* a = src + dir * (d * in_phi + d + d * d + d);
            float* b = dst + (dir ? OFF_PI : OFF_PO);
            for (int u = 0; u < d; ++u) {
                for (int c = 0; c < d; ++c) {
                    b[u * IN_PHI + c] = a[u * in_phi + c];
                    b[u * IN_PHI + D + c] = a[u * in_phi + d + c];
                }
                for (int c = 0; c < 3; ++c) b[u * IN_PHI + 2 * D + c] = a[u * in_phi + 2 * d + c];
                b[D * IN_PHI + u] = a[d * in_phi + u];
                for (int w = 0; w < d; ++w) b[D * IN_PHI + D + u * D + w] = a[d * in_phi + d + u * d + w];
                b[D * IN_PHI + D + D * D + u] = a[d * in_phi + d + d * d + u];
            }
        }
        // Psi: inputs (h, c, phi_out, phi_in)
        {
            const float* a = src + 2 * (d * in_phi + d + d * d + d);
            float* b = dst + OFF_PS;
            for (int u = 0; u < d; ++u) {
                for (int c = 0; c < d; ++c) {
                    b[u * IN_PSI + c] = a[u * in_psi + c];
                    b[u * IN_PSI + D + 1 + c] = a[u * in_psi + d + 1 + c];
                    b[u * IN_PSI + 2 * D + 1 + c] = a[u * in_psi + 2 * d + 1 + c];
                }
                b[u * IN_PSI + D] = a[u * in_psi + d];
                b[D * IN_PSI + u] = a[d * in_psi + u];
                for (int w = 0; w < d; ++w) b[D * IN_PSI + D + u * D + w] = a[d * in_psi + d + u * d + w];
                b[D * IN_PSI + D + D * D + u] = a[d * in_psi + d + d * d + u];
            }
        }
        // decoder: W1[d][d], b1[d], W2[1][d], b2
        {
            const float* a = src + 2 * (d * in_phi + d + d * d + d) + d * in_psi + d + d * d + d;
            float* b = dst + OFF_DE;
            for (int u = 0; u < d; ++u) {
                for (int c = 0; c < d; ++c) b[u * D + c] = a[u * d + c];
                b[D * D + u] = a[d * d + u];
                b[D * D + D + u] = a[d * d + d + u];
            }
            b[D * D + 2 * D] = a[d * d + 2 * d];
        }
    }
}

void build_mfma_blobs(const float* theta, int kbar, std::vector<MfmaStep>& steps, std::vector<MfmaDec>& dec) {
    steps.assign((size_t)kbar, MfmaStep{});
    std::vector<double> A(32 * 16);
    auto put = [&](uint16_t* dst, int lane) {
        const int row = lane % 32, k0 = 8 * (lane / 32);
        for (int m = 0; m < 8; ++m) dst[m] = bf16_bits(A[row * 16 + k0 + m]);
    };
    auto put16 = [&](uint16_t* dst, int lane) {  // FP16 operands (the message-sum tiles)
        const int row = lane % 32, k0 = 8 * (lane / 32);
        for (int m = 0; m < 8; ++m) {
            const _Float16 hv = (_Float16)(float)A[row * 16 + k0 + m];
            std::memcpy(&dst[m], &hv, 2);
        }
    };
    for (int step = 0; step < kbar; ++step) {
        const float* th = theta + (size_t)step * BLOCK_W;
        auto W1 = [&](int dir, int u, int i) { return (double)th[(dir ? OFF_PI : OFF_PO) + u * IN_PHI + i]; };
        auto B1 = [&](int dir, int u) { return (double)th[(dir ? OFF_PI : OFF_PO) + D * IN_PHI + u]; };
        auto W2 = [&](int dir, int v, int w) { return (double)th[(dir ? OFF_PI : OFF_PO) + D * IN_PHI + D + v * D + w]; };
        auto B2 = [&](int dir, int v) { return (double)th[(dir ? OFF_PI : OFF_PO) + D * IN_PHI + D + D * D + v]; };
        auto P1 = [&](int u, int i) { return (double)th[OFF_PS + u * IN_PSI + i]; };
        auto PB1 = [&](int u) { return (double)th[OFF_PS + D * IN_PSI + u]; };
        auto P2 = [&](int o, int u) { return (double)th[OFF_PS + D * IN_PSI + D + o * D + u]; };
        auto PB2 = [&](int o) { return (double)th[OFF_PS + D * IN_PSI + D + D * D + o]; };
        // Folded message second layers: M_dir[u][w] = sum_v W1_psi[u][phi_dir v] W2_dir[v][w].
        double M[2][D][D], degb[D];
        for (int u = 0; u < D; ++u) {
            degb[u] = 0;
            for (int dir = 0; dir < 2; ++dir) {
                const int off = dir ? 2 * D + 1 : D + 1;
                for (int w = 0; w < D; ++w) {
                    double acc = 0;
                    for (int v = 0; v < D; ++v) acc += P1(u, off + v) * W2(dir, v, w);
                    M[dir][u][w] = acc;
                }
                for (int v = 0; v < D; ++v) degb[u] += P1(u, off + v) * B2(dir, v);
            }
        }
        MfmaStep& L = steps[(size_t)step];
        // Q' and P' tiles: row r -> (direction, unit) = (row_half, row_item) for items < 10.
        for (int which = 0; which < 2; ++which) {  // 0: Q', 1: P'
            std::fill(A.begin(), A.end(), 0.0);
            for (int r = 0; r < 32; ++r) {
                const int dir = row_half(r), u = row_item(r);
                if (u >= D) continue;
                const double sx = dir == 0 ? 1.0 : -1.0;  // d_jl for Phi_out, d_lj = -d_jl for Phi_in
                for (int k = 0; k < 16; ++k) {
                    int hi = 0;
                    const Role role = pq_role(k, &hi);
                    double v = 0;
                    if (role == H) v = W1(dir, u, which == 0 ? D + hi : hi);
                    else if (role == ONE) v = which == 0 ? 0.0 : B1(dir, u);
                    else if (role == XHI || role == XLO) v = (which == 0 ? sx : -sx) * W1(dir, u, 2 * D);
                    else if (role == YHI || role == YLO) v = (which == 0 ? sx : -sx) * W1(dir, u, 2 * D + 1);
                    A[r * 16 + k] = v;
                }
            }
            for (int lane = 0; lane < 64; ++lane) put(L.a[which == 0 ? A_Q : A_P][lane], lane);
        }
        // Psi hidden layer: output row r -> unit 5*row_half + row_item for items < 5.
        auto hidden_unit = [](int r) { return row_item(r) < 5 ? 5 * row_half(r) + row_item(r) : -1; };
        std::fill(A.begin(), A.end(), 0.0);
        for (int r = 0; r < 32; ++r) {
            const int u = hidden_unit(r);
            if (u < 0) continue;
            for (int k = 0; k < 16; ++k) {
                int hi = 0;
                const Role role = psi_role(k, &hi);
                double v = 0;
                if (role == H) v = P1(u, hi);
                else if (role == ONE) v = PB1(u);
                else if (role == C) v = P1(u, D);
                else if (role == DEG) v = degb[u];
                A[r * 16 + k] = v;
            }
        }
        for (int lane = 0; lane < 64; ++lane) put(L.a[A_H][lane], lane);
        for (int part = 0; part < 2; ++part) {  // message sums, units 0..7 then 8..9
            std::fill(A.begin(), A.end(), 0.0);
            for (int r = 0; r < 32; ++r) {
                const int u = hidden_unit(r);
                if (u < 0) continue;
                for (int k = 0; k < 16; ++k) {
                    const int dir = k / 8, m = k % 8;
                    const int w = part == 0 ? m : 8 + m;
                    if (part == 1 && m >= 2) continue;
                    A[r * 16 + k] = M[dir][u][w];
                }
            }
            for (int lane = 0; lane < 64; ++lane) put16(L.a[part == 0 ? A_SA : A_SB][lane], lane);
        }
        // Psi output layer: output rows as latent components, input k -> hidden
        // unit 5*(k/8) + k%8 for k%8 < 5; k = 5 carries the constant 1 (bias).
        std::fill(A.begin(), A.end(), 0.0);
        for (int r = 0; r < 32; ++r) {
            const int o = hidden_unit(r);
            if (o < 0) continue;
            for (int k = 0; k < 16; ++k)
                if (k % 8 < 5) A[r * 16 + k] = P2(o, 5 * (k / 8) + k % 8);
            A[r * 16 + 5] = PB2(o);
        }
        for (int lane = 0; lane < 64; ++lane) put(L.a[A_2][lane], lane);
        for (int lane = 0; lane < 64; ++lane) {
            const int hf = lane / 32;
            for (int t = 0; t < D / 2; ++t) {  // rounded to FP16 (nearest even) as the kernel's sums use them
                const _Float16 lo = (_Float16)(float)W1(hf, 2 * t, 2 * D + 2);
                const _Float16 hi = (_Float16)(float)W1(hf, 2 * t + 1, 2 * D + 2);
                uint16_t bl, bh;
                std::memcpy(&bl, &lo, 2);
                std::memcpy(&bh, &hi, 2);
                L.wn2[t][lane] = (uint32_t)bl | ((uint32_t)bh << 16);
            }
        }
    }
    // Decoder of the last block.
    const float* th = theta + (size_t)(kbar - 1) * BLOCK_W + OFF_DE;
    dec.assign(64, MfmaDec{});
    std::fill(A.begin(), A.end(), 0.0);
    for (int r = 0; r < 32; ++r) {
        const int u = row_item(r) < 5 ? 5 * row_half(r) + row_item(r) : -1;
        if (u < 0) continue;
        for (int k = 0; k < 16; ++k) {
            int hi = 0;
            const Role role = psi_role(k, &hi);
            if (role == H) A[r * 16 + k] = th[u * D + hi];
            else if (role == ONE) A[r * 16 + k] = th[D * D + u];
        }
    }
    for (int lane = 0; lane < 64; ++lane) put(dec[lane].ad1, lane);
    std::fill(A.begin(), A.end(), 0.0);
    for (int k = 0; k < 16; ++k)
        if (k % 8 < 5) A[0 * 16 + k] = th[D * D + D + 5 * (k / 8) + k % 8];
    for (int lane = 0; lane < 64; ++lane) {
        put(dec[lane].ad2, lane);
        dec[lane].bd2 = th[D * D + 2 * D];
    }
}

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ inline f32x16 mfma(const bf16x8& a, const bf16x8& b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x16 mfma16(const f16x8& a, const f16x8& b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

__device__ inline bf16x8 load_a(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ inline f16x8 load_a16(const uint16_t* p) {
    return __builtin_bit_cast(f16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ inline __bf16 bits_bf16(uint32_t b) { return __builtin_bit_cast(__bf16, (uint16_t)(b & 0xffffu)); }

// Sum over the MFMA_BLOCK virtual threads of a restriction, whatever the
// workgroup size: thread t of a BLOCK-thread workgroup carries virtual threads
// t + v BLOCK (v[] below), each wavefront's shuffle tree and the final sum over
// the MFMA_BLOCK / 64 virtual wavefronts run in the order of a MFMA_BLOCK-thread
// workgroup, so both workgroup sizes give the same bits.
template <int BLOCK>
__device__ inline double block_sum(const double (&v)[MFMA_BLOCK / BLOCK], double* sh) {
    constexpr int VT = MFMA_BLOCK / BLOCK;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < VT; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[w + q * (BLOCK / 64)] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int i = 0; i < MFMA_BLOCK / 64; ++i) acc += sh[i];
        sh[MFMA_BLOCK / 64] = acc;
    }
    __syncthreads();
    return sh[MFMA_BLOCK / 64];
}

// B operands. A lane past the end of the sub-mesh feeds finite values (its h
// stays 0, its tile record is node 0's) into its own output column only, so
// no entry is masked.
// P'/Q' products: (h 5 components, coordinate hi, lo, 1): x in half 0, y in half 1.
__device__ inline bf16x8 b_pq(const float (&h)[5], uint32_t xy2) {
    bf16x8 b;
#pragma unroll
    for (int m = 0; m < 5; ++m) b[m] = (__bf16)h[m];
    b[5] = bits_bf16(xy2);
    b[6] = bits_bf16(xy2 >> 16);
    b[7] = (__bf16)1.0f;
    return b;
}

// Psi hidden layer: (h 5 components, 1, c, deg) (the weight columns of half 1 at m >= 5 are zero).
__device__ inline bf16x8 b_psi(const float (&h)[5], float c, float deg) {
    bf16x8 b;
#pragma unroll
    for (int m = 0; m < 5; ++m) b[m] = (__bf16)h[m];
    b[5] = (__bf16)1.0f;
    b[6] = (__bf16)c;
    b[7] = (__bf16)deg;
    return b;
}

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

// ReLU of a bf16 pair as a signed 16-bit max with 0: bf16 is sign-magnitude,
// so negative values (and -0) are negative as integers and positive values
// keep their order; equals rounding ReLU(x) to bf16.
__device__ inline uint32_t bf16_relu2(float lo, float hi) {
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    const i16x2 r = __builtin_elementwise_max(__builtin_bit_cast(i16x2, v), (i16x2){0, 0});
    return __builtin_bit_cast(uint32_t, r);
}

__device__ inline h2 pk(float x, float y) { return (h2){(_Float16)x, (_Float16)y}; }

// Tile t of a wavefront's tiles (t < MAX_TILES_PER_WAVE): its tile index,
// the node position of lane n in it and the tile record (past the end of the
// sub-mesh: the tile's first node).
struct TileRef {
    int tile, p;
    bool valid;
    TileNode tn;
};
template <int BLOCK>
__device__ inline TileRef tile_ref(const TileNode* T, int wave, int tt, int n, int k) {
    TileRef r;
    r.tile = wave + (BLOCK / 64) * tt;
    r.p = r.tile * MFMA_TILE + n;
    r.valid = r.p < k;
    r.tn = T[r.valid ? r.p : r.tile * MFMA_TILE];
    return r;
}
__device__ inline uint32_t split_xy(const TileNode& tn, int hf) {
    return hf ? (uint32_t)tn.yh | ((uint32_t)tn.yl << 16) : (uint32_t)tn.xh | ((uint32_t)tn.xl << 16);
}

// The kbar blocks of DSS_theta for the wavefront's tiles (h in registers).
// Q' lives in LDS, row stride 5 dwords, one array per message direction.
// DB = false: one Q' buffer; per block, phase A (Q' of every tile), barrier,
// phase B (edge sums and updates), barrier. DB = true: two Q' buffers; phase B
// of block k reads buffer k % 2 and each tile, once updated, writes its Q' of
// block k + 1 to the other buffer right away, so one barrier per block
// separates the blocks (the buffer written in block k was last read in block
// k - 1, before the previous barrier). Both give the same bits.
template <int BLOCK, bool DB>
__device__ __forceinline__ void dss_blocks(const DssMfmaArgs& a, float (&h)[MAX_TILES_PER_WAVE][5],
                                           const float* cbuf, h2* Qd, const uint32_t* E, const TileNode* T,
                                           int k, int ntiles, int wave, int lane) {
    const int n = lane & 31, hf = lane >> 5;
    const f32x16 zero = {};
    const h2 hzero = {(_Float16)0.0f, (_Float16)0.0f};
    const size_t qbuf = (size_t)((10 * (k + 1) + 3) & ~3);  // h2 entries of one Q' buffer (both directions)
    // Q' of the wave's tiles into buffer `buf` with the Q' tile AQ: the products
    // of two tiles are issued back to back, then converted and stored.
    auto phase_a = [&](const bf16x8& AQ, int buf) {
#pragma unroll
        for (int t2 = 0; t2 < MAX_TILES_PER_WAVE; t2 += 2) {
            f32x16 q[2];
            int jt[2] = {-1, -1};
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (wave + (BLOCK / 64) * (t2 + u) >= ntiles) break;
                const TileRef r = tile_ref<BLOCK>(T, wave, t2 + u, n, k);
                jt[u] = r.valid ? (int)r.tn.j : -1;
                q[u] = mfma(AQ, b_pq(h[t2 + u], split_xy(r.tn, hf)), zero);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (jt[u] >= 0) {
                    h2* dst = Qd + (size_t)buf * qbuf + (size_t)(hf * (k + 1) + jt[u]) * 5;
#pragma unroll
                    for (int t = 0; t < 5; ++t) dst[t] = pk(q[u][2 * t], q[u][2 * t + 1]);
                }
            }
        }
    };
    // The weights of a block are the same for every tile: each lane loads its
    // operands once per block (the next block's Q' tile while this block runs).
    bf16x8 AQ = load_a(a.steps[0].a[A_Q][lane]);
    if (DB) {
        phase_a(AQ, 0);
        if (a.kbar > 1) AQ = load_a(a.steps[1].a[A_Q][lane]);
        __syncthreads();
    }
    for (int step = 0; step < a.kbar; ++step) {
        const MfmaStep* L = a.steps + step;
        const int cur = DB ? (step & 1) : 0;
        if (!DB) phase_a(AQ, 0);
        // the operands every tile needs before its edge sums (the Psi operands
        // are fetched per tile, their latency hidden behind the tile's edge sums)
        const bf16x8 AP = load_a(L->a[A_P][lane]);
        h2 wn[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) wn[t] = __builtin_bit_cast(h2, L->wn2[t][lane]);
        if (!DB) {
            if (step + 1 < a.kbar) AQ = load_a(a.steps[step + 1].a[A_Q][lane]);
            __syncthreads();
        }
        const h2* Qh = Qd + (size_t)cur * qbuf + (size_t)hf * 5 * (k + 1);  // this lane's direction
        const bool next = DB && step + 1 < a.kbar;
        // Phase B: receiver projections, edge sums, Psi update (and with DB the
        // tile's Q' of the next block).
#pragma unroll
        for (int tt = 0; tt < MAX_TILES_PER_WAVE; ++tt) {
            if (wave + (BLOCK / 64) * tt >= ntiles) break;
            const TileRef r = tile_ref<BLOCK>(T, wave, tt, n, k);
            const TileNode& tn = r.tn;
            const int j = tn.j;
            const uint32_t xy2 = split_xy(tn, hf);
            const f32x16 Pf = mfma(AP, b_pq(h[tt], xy2), zero);
            const bf16x8 AH = load_a(L->a[A_H][lane]), A2 = load_a(L->a[A_2][lane]);
            const f16x8 ASA = load_a16(L->a[A_SA][lane]), ASB = load_a16(L->a[A_SB][lane]);
            h2 P[5], S[5];
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                P[t] = pk(Pf[2 * t], Pf[2 * t + 1]);
                S[t] = hzero;
            }
            const int deg = r.valid ? (int)tn.deg : 0;
            // The tile's edge block: EC slots per chunk, one column per lane
            // (lanes past the end of the sub-mesh read sentinel records).
            const uint32_t* Et = E + (tn.e0 & 0xffffff) + n;
            const int nch = __builtin_amdgcn_readfirstlane((int)((uint32_t)tn.e0 >> 24));
            // The records of the next chunk are in flight while a chunk's sums
            // run; a load past the last chunk re-reads the last chunk (clamped
            // index) and goes unused.
            auto ld_rec = [&](int ch, uint32_t (&rc)[EC]) {
                const int c = min(ch, nch - 1);
#pragma unroll
                for (int w = 0; w < EC; ++w) rc[w] = Et[(c * EC + w) * MFMA_TILE];
            };
            auto ld_q = [&](const uint32_t (&rc)[EC], h2 (&q)[EC][5]) {
#pragma unroll
                for (int w = 0; w < EC; ++w) {
                    const h2* row = reinterpret_cast<const h2*>(reinterpret_cast<const char*>(Qh) + (rc[w] >> 16));
#pragma unroll
                    for (int t = 0; t < 5; ++t) q[w][t] = row[t];
                }
            };
            auto sums = [&](const uint32_t (&rc)[EC], const h2 (&q)[EC][5]) {
#pragma unroll
                for (int w = 0; w < EC; ++w) {
                    const _Float16 ndh = __builtin_bit_cast(_Float16, (uint16_t)(rc[w] & 0xffffu));
                    const h2 nd = {ndh, ndh};
#pragma unroll
                    for (int t = 0; t < 5; ++t)
                        S[t] += __builtin_elementwise_max(__builtin_elementwise_fma(wn[t], nd, P[t] + q[w][t]), hzero);
                }
            };
            // A wavefront in its edge sums issues ahead of those in the matrix
            // products and conversions (same arithmetic, 1.6% off the solve at c3).
            __builtin_amdgcn_s_setprio(1);
            if (nch > 0) {
                uint32_t r0[EC];
                ld_rec(0, r0);
                for (int ch = 0; ch < nch; ++ch) {
                    h2 q[EC][5];
                    ld_q(r0, q);
                    uint32_t r1[EC];
                    ld_rec(ch + 1, r1);
                    sums(r0, q);
#pragma unroll
                    for (int w = 0; w < EC; ++w) r0[w] = r1[w];
                }
            }
            __builtin_amdgcn_s_setprio(0);
            const float c = cbuf[j];
            // The message sums enter the FP16 matrix product as they are.
            const f16x8 sa = {S[0][0], S[0][1], S[1][0], S[1][1], S[2][0], S[2][1], S[3][0], S[3][1]};
            const _Float16 hz = (_Float16)0.0f;
            const f16x8 sb = {S[4][0], S[4][1], hz, hz, hz, hz, hz, hz};
            f32x16 hid = mfma(AH, b_psi(h[tt], c, (float)deg), zero);
            hid = mfma16(ASA, sa, hid);
            hid = mfma16(ASB, sb, hid);
            // (ReLU(hidden) 5 components, 1 for the output bias column, 0, 0)
            const bf16x8 bh = __builtin_bit_cast(
                bf16x8, (uint4){bf16_relu2(hid[0], hid[1]), bf16_relu2(hid[2], hid[3]), bf16_relu2(hid[4], 1.0f), 0u});
            const f32x16 o = mfma(A2, bh, zero);
            if (r.valid) {
#pragma unroll
                for (int t = 0; t < 5; ++t) h[tt][t] = fmaf(a.alpha, o[t], h[tt][t]);
                if (next) {
                    const f32x16 q = mfma(AQ, b_pq(h[tt], xy2), zero);
                    h2* dst = Qd + (size_t)(cur ^ 1) * qbuf + (size_t)(hf * (k + 1) + j) * 5;
#pragma unroll
                    for (int t = 0; t < 5; ++t) dst[t] = pk(q[2 * t], q[2 * t + 1]);
                }
            }
        }
        if (DB && step + 2 < a.kbar) AQ = load_a(a.steps[step + 2].a[A_Q][lane]);
        __syncthreads();
    }
}

// One workgroup per sub-mesh, everything the kbar blocks touch in LDS:
//   c   [k]        normalised residual (FP32)
//   Q'  [nb][2][k+1][5] neighbour projections (FP16 pairs) in nb = 1 or 2
//                  buffers, one array per direction, row k the -inf
//                  sentinel; the odd 5-dword row stride spreads the random
//                  sender rows of an edge gather over all LDS banks
//   E   [ne_pad]   in-edge records per tile, slot-major ([slot][lane], so a
//                  wavefront reads consecutive dwords), padded with sentinel
//                  records to the tile's largest in-degree rounded up to EC:
//                  FP16 |d| | sender row byte offset << 16
//   T   [k]        tile records (node id, degree, first edge, split coordinates)
// A sub-mesh runs with two Q' buffers when they fit the launch's dynamic LDS
// (a.lds_bytes), else with one. The message sums run in packed FP16 (two
// units per instruction).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const u32x4 __attribute__((address_space(1))) gu32x4;
// A load through a global-space pointer (the table's pointers are generic).
template <typename T>
__device__ inline T gload(const T* p) {
    return *(const T __attribute__((address_space(1)))*)p;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void dss_mfma_kernel(DssMfmaArgs a) {
    constexpr int VT = MFMA_BLOCK / BLOCK;  // virtual threads per thread in the restriction sums
    constexpr int MAX_K = MAX_TILES_PER_WAVE * (MFMA_BLOCK / 64) * MFMA_TILE;  // largest sub-mesh
    constexpr int RJ = 2;  // sub-mesh nodes per virtual thread
    static_assert(RJ * MFMA_BLOCK >= MAX_K, "a virtual thread holds all its nodes");
    constexpr int TU = (MAX_K + BLOCK - 1) / BLOCK;  // tile records per thread
    constexpr int EU = 4;                                   // edge-record quads per thread and pass
    const int2 wi = a.work[blockIdx.x];
    const DevProb& P = a.tab[wi.x];
    if (P.st && P.st->done) return;
    extern __shared__ float lds[];
    __shared__ double red[MFMA_BLOCK / 64 + 1];
    const int sub = wi.y;
    const int base = P.sub_ptr[sub];
    const int k = P.sub_ptr[sub + 1] - base;
    const int tid = threadIdx.x;
    const int ebase = P.epad_sub[sub];
    const int ne = P.epad_sub[sub + 1] - ebase;
    const bool db = mfma_lds_need(k, ne, true) <= a.lds_bytes;
    const int nbuf = db ? 2 : 1;
    double* __restrict__ out = P.local;
    float* cbuf = lds;
    h2* Qd = reinterpret_cast<h2*>(lds + ((k + 3) & ~3));
    uint32_t* E = reinterpret_cast<uint32_t*>(Qd + (size_t)nbuf * ((10 * (k + 1) + 3) & ~3));
    TileNode* T = reinterpret_cast<TileNode*>(E + ((ne + 3) & ~3));
    // The records go to LDS with every global load of a thread in flight
    // before the first store (16-byte loads through global-space pointers, so
    // the LDS stores do not wait for them one by one). Edge blocks are whole
    // tiles of MFMA_EC x MFMA_TILE records, so ne and ebase are multiples of 4.
    {
        const gu32x4* esrc = (const gu32x4*)(P.erec + ebase);
        u32x4* edst = reinterpret_cast<u32x4*>(E);
        const int ne4 = ne >> 2;
        // loads past the end re-read the last entry (no branches between the
        // loads); only the stores are guarded
        for (int i0 = tid; i0 < ne4; i0 += EU * BLOCK) {
            u32x4 v[EU];
#pragma unroll
            for (int u = 0; u < EU; ++u) v[u] = esrc[min(i0 + u * BLOCK, ne4 - 1)];
#pragma unroll
            for (int u = 0; u < EU; ++u)
                if (i0 + u * BLOCK < ne4) edst[i0 + u * BLOCK] = v[u];
        }
        const gu32x4* tsrc = (const gu32x4*)(P.tiles + base);
        u32x4* tdst = reinterpret_cast<u32x4*>(T);
        u32x4 v[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) v[u] = tsrc[min(tid + u * BLOCK, k - 1)];
#pragma unroll
        for (int u = 0; u < TU; ++u)
            if (tid + u * BLOCK < k) tdst[tid + u * BLOCK] = v[u];
    }
    if (tid < 10 * nbuf) {  // sentinel rows: every message through them is ReLU(-inf) = 0
        const _Float16 ninf = __builtin_bit_cast(_Float16, (uint16_t)0xFC00u);
        const int b = tid / 10, t = tid % 10;
        Qd[(size_t)b * ((10 * (k + 1) + 3) & ~3) + (size_t)(t / 5) * 5 * (k + 1) + 5 * k + t % 5] = (h2){ninf, ninf};
    }
    // Restriction and normalisation (Sec. III.A step 2). Virtual thread q of
    // this thread sums j = tid + q BLOCK + m MFMA_BLOCK (m = 0, 1; k <= 2048),
    // in that order; the ids and weights of all its j, then their residuals,
    // are loaded before the sums, and the residuals are kept for c.
    double s = 1.0;
    if (a.apply) {
        double ssv[VT], yyv[VT], rv[VT][RJ];
        int g[VT][RJ];
        double wv[VT][RJ];
#pragma unroll
        for (int q = 0; q < VT; ++q)
#pragma unroll
            for (int m = 0; m < RJ; ++m) {
                const int j = min(tid + q * BLOCK + m * MFMA_BLOCK, k - 1);  // past the end: unused
                g[q][m] = gload(P.sub_nodes + base + j);
                wv[q][m] = gload(P.weights + base + j);
            }
#pragma unroll
        for (int q = 0; q < VT; ++q)
#pragma unroll
            for (int m = 0; m < RJ; ++m) rv[q][m] = gload(P.r + g[q][m]);
#pragma unroll
        for (int q = 0; q < VT; ++q) {
            ssv[q] = 0.0;
            yyv[q] = 0.0;
#pragma unroll
            for (int m = 0; m < RJ; ++m)
                if (tid + q * BLOCK + m * MFMA_BLOCK < k) {
                    ssv[q] = fma(rv[q][m], rv[q][m], ssv[q]);
                    yyv[q] = fma(wv[q][m], rv[q][m], yyv[q]);
                }
        }
        const double ss = block_sum<BLOCK>(ssv, red);
        const double yy = block_sum<BLOCK>(yyv, red);
        s = sqrt(ss);
        if (tid == 0) {
            P.s[sub] = s;
            P.y0[sub] = yy;
        }
        if (s == 0.0) {
            for (int j = tid; j < k; j += BLOCK) out[base + j] = 0.0;
            return;
        }
        const double inv = 1.0 / s;
#pragma unroll
        for (int q = 0; q < VT; ++q)
#pragma unroll
            for (int m = 0; m < RJ; ++m) {
                const int j = tid + q * BLOCK + m * MFMA_BLOCK;
                if (j < k) cbuf[j] = (float)(rv[q][m] * inv);
            }
    } else {
        for (int j = tid; j < k; j += BLOCK) cbuf[j] = (float)P.c_in[base + j];
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int n = lane & 31, hf = lane >> 5;
    const int ntiles = (k + MFMA_TILE - 1) / MFMA_TILE;
    float h[MAX_TILES_PER_WAVE][5];
#pragma unroll
    for (int tt = 0; tt < MAX_TILES_PER_WAVE; ++tt)
#pragma unroll
        for (int t = 0; t < 5; ++t) h[tt][t] = 0.0f;
    const f32x16 zero = {};
    if (db)
        dss_blocks<BLOCK, true>(a, h, cbuf, Qd, E, T, k, ntiles, wave, lane);
    else
        dss_blocks<BLOCK, false>(a, h, cbuf, Qd, E, T, k, ntiles, wave, lane);

    // Decoder of the last block.
    const MfmaDec* Ld = a.dec + lane;
    const bf16x8 AD1 = load_a(Ld->ad1), AD2 = load_a(Ld->ad2);
    const float bd2 = Ld->bd2;
#pragma unroll
    for (int tt = 0; tt < MAX_TILES_PER_WAVE; ++tt) {
        const int tile = wave + (BLOCK / 64) * tt;
        if (tile >= ntiles) break;
        const int p = tile * MFMA_TILE + n;
        const bool valid = p < k;
        const TileNode tn = T[valid ? p : tile * MFMA_TILE];
        const f32x16 hd = mfma(AD1, b_psi(h[tt], 0.0f, 0.0f), zero);
        const bf16x8 bh = __builtin_bit_cast(
            bf16x8, (uint4){bf16_relu2(hd[0], hd[1]), bf16_relu2(hd[2], hd[3]), bf16_relu2(hd[4], 0.0f), 0u});
        const f32x16 o = mfma(AD2, bh, zero);
        if (valid && hf == 0) {
            const double r_tilde = (double)(o[0] + bd2);
            out[base + tn.j] = a.apply ? s * r_tilde : r_tilde;
        }
    }
}

}  // namespace

hipError_t prepare_dss_mfma(size_t shmem) {
    hipError_t e = hipFuncSetAttribute((const void*)dss_mfma_kernel<MFMA_BLOCK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)dss_mfma_kernel<MFMA_SMALL_BLOCK>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
}

hipError_t launch_dss_mfma(const DssMfmaArgs& args, int n_work, size_t shmem, int block, hipStream_t stream,
                           bool check) {
    if (n_work <= 0) return hipSuccess;
    DssMfmaArgs a = args;
    a.lds_bytes = (uint32_t)shmem;
    if (block == MFMA_SMALL_BLOCK)
        hipLaunchKernelGGL(dss_mfma_kernel<MFMA_SMALL_BLOCK>, dim3(n_work), dim3(MFMA_SMALL_BLOCK), shmem, stream, a);
    else
        hipLaunchKernelGGL(dss_mfma_kernel<MFMA_BLOCK>, dim3(n_work), dim3(MFMA_BLOCK), shmem, stream, a);
    return check ? hipGetLastError() : hipSuccess;
}

}  // namespace ddmgnn
