// Training of DSS_theta (Sec. III.B, Sec. IV.B): the loss is the residual loss
// L_res of Sec. II.B (squared residual of the local system A_i u = c) of the
// decoded state of every block, summed over the kbar blocks. One workgroup
// takes one local problem (a sub-mesh and its right-hand side c), runs the
// forward pass keeping the latent states H^0..H^kbar, then walks the blocks
// backwards: it recomputes a block's intermediates from H^{k-1}, propagates
// the gradient and writes the block's weight gradient.
//
// Weight gradients are sums over the nodes of per-node outer products. The
// per-edge terms of the first message layer reduce to per-node sums first:
// with g_e the gradient of edge e's hidden pre-activation (the receiver's
// back-propagated message gradient masked by the edge's ReLU),
//   dW1[:, h_j] = sum_j (sum_{e into j} g_e) h_j^T,
//   dW1[:, h_l] = sum_l (sum_{e out of l} g_e) h_l^T,
// and the coordinate and |d| columns take per-receiver sums of g_e d_e and
// g_e |d_e|. Every sum runs in a fixed order, so the gradient is
// deterministic. Arithmetic is FP32 with explicit fused multiply-adds, so a
// recomputed pre-activation has the bits of the first evaluation and the
// ReLU masks agree between the receiver and the sender passes.
#include "device.h"

namespace ddmgnn {

namespace {

constexpr int TB = TRAIN_BLOCK;
constexpr int F_PHI = 2 * D + 3, F_PSI = 3 * D + 1;
constexpr int O_PO = 0;
constexpr int O_PI = O_PO + D * F_PHI + D + D * D + D;
constexpr int O_PS = O_PI + D * F_PHI + D + D * D + D;
constexpr int O_DE = O_PS + D * F_PSI + D + D * D + D;
static_assert(O_DE + D * D + D + D + 1 == TRAIN_NWB, "weights per block");

// Per-node arrays of D floats in a sample's scratch, after the state history.
enum Arr {
    PO, PI, QO, QI,        // receiver and sender parts of the message hidden layers
    MO, MI,                // sums of the message hidden activations
    FO, FI,                // messages phi_out, phi_in
    ZP, UP,                // Psi hidden layer before and after ReLU
    ZD, UD,                // decoder hidden layer before and after ReLU
    GZD, GPS, GZ,          // gradients: decoder hidden, Psi output, Psi hidden
    GFO, GFI, GMO, GMI,    // gradients: messages, message hidden sums
    GRO, GRI, GSO, GSI,    // per receiver / per sender sums of edge gradients
    NO, NI, DXO, DXI, DYO, DYI,  // per receiver sums of g_e |d_e|, g_e dx_e, g_e dy_e
    GH, GHN,               // gradient of the loss w.r.t. H^k and H^{k-1}
    N_ARR
};
// Per-node scalars after those: decoded r_hat, residual rho, its gradient.
enum Sca { SR, SRHO, SGR, N_SCA };

}  // namespace

int64_t train_scratch_floats(int kbar, int64_t k) { return ((int64_t)(kbar + 1 + N_ARR) * D + N_SCA) * k; }

namespace {

struct Sample {
    float* base;
    int64_t k;
    __device__ float* hist(int s) const { return base + (int64_t)s * k * D; }
    __device__ float* arr(int kbar, int a) const { return base + (int64_t)(kbar + 1 + a) * k * D; }
    __device__ float* sca(int kbar, int a) const { return base + (int64_t)(kbar + 1 + N_ARR) * k * D + (int64_t)a * k; }
};

// Hidden pre-activation of unit u of a message MLP for one edge: receiver part
// + sender part + coordinate and length terms (sx = -1 flips d for Phi_in).
__device__ inline float pre(float pr, float qs, const float* w1u, float sx, float dx, float dy, float nd) {
    float t = pr + qs;
    t = fmaf(sx * w1u[2 * D], dx, t);
    t = fmaf(sx * w1u[2 * D + 1], dy, t);
    return fmaf(w1u[2 * D + 2], nd, t);
}

// Receiver (b1 + W1[:, h_j] h) and sender (W1[:, h_l] h) parts of one message MLP.
__device__ inline void pq(const float* w, const float* h, float* p, float* q) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const float* r = w + u * F_PHI;
        float a = w[D * F_PHI + u], b = 0.0f;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            a = fmaf(r[i], h[i], a);
            b = fmaf(r[D + i], h[i], b);
        }
        p[u] = a;
        q[u] = b;
    }
}

__device__ inline void ld(const float* src, float* dst) {
#pragma unroll
    for (int i = 0; i < D; ++i) dst[i] = src[i];
}
__device__ inline void st(float* dst, const float* src) {
#pragma unroll
    for (int i = 0; i < D; ++i) dst[i] = src[i];
}

struct Edge {
    float dx, dy, nd;
};
// d = x_send - x_recv from the FP64 coordinates of the two slots.
__device__ inline Edge edge(const TrainArgs& a, int64_t b, int recv, int send, int t) {
    Edge e;
    e.dx = (float)(a.xy64[2 * (b + send)] - a.xy64[2 * (b + recv)]);
    e.dy = (float)(a.xy64[2 * (b + send) + 1] - a.xy64[2 * (b + recv) + 1]);
    e.nd = a.edge_nd[t];
    return e;
}

__device__ inline double block_sum_d(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double acc = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < TB / 64; ++i) acc += sh[i];
    return acc;
}

// One block's forward for node j from H = H^{k-1}: messages, Psi, new state.
// With keep, the intermediates are stored for the backward pass.
__device__ __noinline__ void block_node(const TrainArgs& a, const Sample& S, const float* w, const float* H, float* Hn,
                                  const float* cs, int64_t b, int j, bool keep) {
    const int kb = a.kbar;
    float po[D], pi[D], mo[D], mi[D];
    ld(S.arr(kb, PO) + j * D, po);
    ld(S.arr(kb, PI) + j * D, pi);
#pragma unroll
    for (int u = 0; u < D; ++u) mo[u] = mi[u] = 0.0f;
    const int e0 = a.edge_ptr[b + j], e1 = a.edge_ptr[b + j + 1];
    for (int t = e0; t < e1; ++t) {
        const int l = a.edge_src[t];
        const Edge e = edge(a, b, j, l, t);
        const float* qo = S.arr(kb, QO) + l * D;
        const float* qi = S.arr(kb, QI) + l * D;
#pragma unroll
        for (int u = 0; u < D; ++u) {
            mo[u] += fmaxf(pre(po[u], qo[u], w + O_PO + u * F_PHI, 1.0f, e.dx, e.dy, e.nd), 0.0f);
            mi[u] += fmaxf(pre(pi[u], qi[u], w + O_PI + u * F_PHI, -1.0f, e.dx, e.dy, e.nd), 0.0f);
        }
    }
    const float deg = (float)(e1 - e0);
    float x[F_PSI];  // (h, c, phi_out, phi_in)
    ld(H + j * D, x);
    x[D] = cs[j];
#pragma unroll
    for (int v = 0; v < D; ++v) {
        const float* w2o = w + O_PO + D * F_PHI + D + v * D;
        const float* w2i = w + O_PI + D * F_PHI + D + v * D;
        float fo = deg * w[O_PO + D * F_PHI + D + D * D + v], fi = deg * w[O_PI + D * F_PHI + D + D * D + v];
#pragma unroll
        for (int u = 0; u < D; ++u) {
            fo = fmaf(w2o[u], mo[u], fo);
            fi = fmaf(w2i[u], mi[u], fi);
        }
        x[D + 1 + v] = fo;
        x[2 * D + 1 + v] = fi;
    }
    float z[D], hu[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const float* r = w + O_PS + u * F_PSI;
        float acc = w[O_PS + D * F_PSI + u];
#pragma unroll
        for (int i = 0; i < F_PSI; ++i) acc = fmaf(r[i], x[i], acc);
        z[u] = acc;
        hu[u] = fmaxf(acc, 0.0f);
    }
    if (keep) {
        st(S.arr(kb, MO) + j * D, mo);
        st(S.arr(kb, MI) + j * D, mi);
        st(S.arr(kb, FO) + j * D, x + D + 1);
        st(S.arr(kb, FI) + j * D, x + 2 * D + 1);
        st(S.arr(kb, ZP) + j * D, z);
        st(S.arr(kb, UP) + j * D, hu);
    } else {
        float hn[D];
#pragma unroll
        for (int o = 0; o < D; ++o) {
            const float* r = w + O_PS + D * F_PSI + D + o * D;
            float acc = w[O_PS + D * F_PSI + D + D * D + o];
#pragma unroll
            for (int u = 0; u < D; ++u) acc = fmaf(r[u], hu[u], acc);
            hn[o] = fmaf(a.alpha, acc, x[o]);
        }
        st(Hn + j * D, hn);
    }
}

// Weight gradients as sums over node tiles staged in LDS. A tile holds, for
// CH nodes, every per-node quantity a gradient entry multiplies: rows of CH
// values (padded to CHP so that the rows of one wavefront's entries fall on
// different banks), D rows per vector quantity, then the scalars c, dL/dr_hat
// and the in-degree.
constexpr int CH = 32;
constexpr int CHP = CH + 1;
enum TSlot { T_HP, T_HC, T_GRO, T_GSO, T_DXO, T_DYO, T_NO, T_GFO, T_MO, T_GRI, T_GSI, T_DXI, T_DYI, T_NI, T_GFI,
             T_MI, T_GZ, T_FO, T_FI, T_GPS, T_UP, T_GZD, T_UD, N_TV };
constexpr int ROW_C = N_TV * D, ROW_GR = ROW_C + 1, ROW_DEG = ROW_C + 2, N_ROWS = ROW_C + 3;
constexpr int ROW_ONE = -1;

__device__ inline const float* tile_src(const Sample& S, int kb, int blk, int slot) {
    switch (slot) {
        case T_HP: return S.hist(blk);
        case T_HC: return S.hist(blk + 1);
        case T_GRO: return S.arr(kb, GRO);
        case T_GSO: return S.arr(kb, GSO);
        case T_DXO: return S.arr(kb, DXO);
        case T_DYO: return S.arr(kb, DYO);
        case T_NO: return S.arr(kb, NO);
        case T_GFO: return S.arr(kb, GFO);
        case T_MO: return S.arr(kb, MO);
        case T_GRI: return S.arr(kb, GRI);
        case T_GSI: return S.arr(kb, GSI);
        case T_DXI: return S.arr(kb, DXI);
        case T_DYI: return S.arr(kb, DYI);
        case T_NI: return S.arr(kb, NI);
        case T_GFI: return S.arr(kb, GFI);
        case T_MI: return S.arr(kb, MI);
        case T_GZ: return S.arr(kb, GZ);
        case T_FO: return S.arr(kb, FO);
        case T_FI: return S.arr(kb, FI);
        case T_GPS: return S.arr(kb, GPS);
        case T_UP: return S.arr(kb, UP);
        case T_GZD: return S.arr(kb, GZD);
        default: return S.arr(kb, UD);
    }
}

// Gradient entry e of a block = sign * sum_j tile[ra][j] * tile[rb][j] (rb = ROW_ONE: 1).
struct Ent {
    int ra, rb;
    float sign;
};
__device__ inline int row(int slot, int comp) { return slot * D + comp; }
__device__ Ent decode(int e) {
    if (e < O_PS) {
        const bool out = e < O_PI;
        const int r = e - (out ? O_PO : O_PI);
        const int GR_ = out ? T_GRO : T_GRI, GS_ = out ? T_GSO : T_GSI, DX_ = out ? T_DXO : T_DXI;
        const int DY_ = out ? T_DYO : T_DYI, N_ = out ? T_NO : T_NI, GF_ = out ? T_GFO : T_GFI;
        const int M_ = out ? T_MO : T_MI;
        const float sg = out ? 1.0f : -1.0f;  // Phi_in sees d_lj = -d_jl
        if (r < D * F_PHI) {
            const int u = r / F_PHI, i = r % F_PHI;
            if (i < D) return {row(GR_, u), row(T_HP, i), 1.0f};
            if (i < 2 * D) return {row(GS_, u), row(T_HP, i - D), 1.0f};
            if (i == 2 * D) return {row(DX_, u), ROW_ONE, sg};
            if (i == 2 * D + 1) return {row(DY_, u), ROW_ONE, sg};
            return {row(N_, u), ROW_ONE, 1.0f};
        }
        if (r < D * F_PHI + D) return {row(GR_, r - D * F_PHI), ROW_ONE, 1.0f};
        if (r < D * F_PHI + D + D * D) {
            const int q = r - D * F_PHI - D;
            return {row(GF_, q / D), row(M_, q % D), 1.0f};
        }
        return {row(GF_, r - D * F_PHI - D - D * D), ROW_DEG, 1.0f};
    }
    if (e < O_DE) {
        const int r = e - O_PS;
        if (r < D * F_PSI) {
            const int u = r / F_PSI, i = r % F_PSI;
            if (i < D) return {row(T_GZ, u), row(T_HP, i), 1.0f};
            if (i == D) return {row(T_GZ, u), ROW_C, 1.0f};
            if (i < 2 * D + 1) return {row(T_GZ, u), row(T_FO, i - D - 1), 1.0f};
            return {row(T_GZ, u), row(T_FI, i - 2 * D - 1), 1.0f};
        }
        if (r < D * F_PSI + D) return {row(T_GZ, r - D * F_PSI), ROW_ONE, 1.0f};
        if (r < D * F_PSI + D + D * D) {
            const int q = r - D * F_PSI - D;
            return {row(T_GPS, q / D), row(T_UP, q % D), 1.0f};
        }
        return {row(T_GPS, r - D * F_PSI - D - D * D), ROW_ONE, 1.0f};
    }
    const int r = e - O_DE;
    if (r < D * D) return {row(T_GZD, r / D), row(T_HC, r % D), 1.0f};
    if (r < D * D + D) return {row(T_GZD, r - D * D), ROW_ONE, 1.0f};
    if (r < D * D + 2 * D) return {ROW_GR, row(T_UD, r - D * D - D), 1.0f};
    return {ROW_GR, ROW_ONE, 1.0f};
}

constexpr int GR_ROUNDS = (TRAIN_NWB + TB - 1) / TB;

// Block `blk`'s weight gradient for this thread's entries (e = tid + r TB), summed
// over the nodes in ascending order, tile by tile.
__device__ void block_grad(const TrainArgs& a, const Sample& S, const float* cs, int64_t b, int blk, float* tile,
                           float* gout) {
    const int kb = a.kbar, k = (int)S.k, tid = threadIdx.x;
    Ent ent[GR_ROUNDS];
    float acc[GR_ROUNDS];
#pragma unroll
    for (int r = 0; r < GR_ROUNDS; ++r) {
        const int e = tid + r * TB;
        ent[r] = e < TRAIN_NWB ? decode(e) : Ent{0, ROW_ONE, 0.0f};
        acc[r] = 0.0f;
    }
    for (int j0 = 0; j0 < k; j0 += CH) {
        __syncthreads();
        for (int idx = tid; idx < N_TV * CH * D; idx += TB) {
            const int slot = idx / (CH * D), rem = idx % (CH * D), n = rem / D, comp = rem % D;
            const int j = j0 + n;
            tile[(slot * D + comp) * CHP + n] = j < k ? tile_src(S, kb, blk, slot)[j * D + comp] : 0.0f;
        }
        for (int idx = tid; idx < 3 * CH; idx += TB) {
            const int which = idx / CH, n = idx % CH, j = j0 + n;
            float v = 0.0f;
            if (j < k)
                v = which == 0 ? cs[j]
                               : which == 1 ? S.sca(kb, SGR)[j]
                                            : (float)(a.edge_ptr[b + j + 1] - a.edge_ptr[b + j]);
            tile[(ROW_C + which) * CHP + n] = v;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < GR_ROUNDS; ++r) {
            const float* A = tile + ent[r].ra * CHP;
            float x = acc[r];
            if (ent[r].rb == ROW_ONE) {
                for (int n = 0; n < CH; ++n) x += A[n];
            } else {
                const float* B = tile + ent[r].rb * CHP;
                for (int n = 0; n < CH; ++n) x = fmaf(A[n], B[n], x);
            }
            acc[r] = x;
        }
    }
#pragma unroll
    for (int r = 0; r < GR_ROUNDS; ++r) {
        const int e = tid + r * TB;
        if (e < TRAIN_NWB) gout[e] = ent[r].sign * acc[r];
    }
}

// Back through the decoder of H^k, Psi and the second message layers for node j.
__device__ __noinline__ void psi_back_node(const TrainArgs& a, const Sample& S, const float* w, const float* cs,
                                           int64_t b, int j) {
    const int kb = a.kbar;
    float acc = 0.0f;  // (A_i^T rho)_j = (A_i rho)_j: A_i is symmetric
    for (int q = a.lm_ptr[b + j]; q < a.lm_ptr[b + j + 1]; ++q)
        acc = fmaf(a.lm_val[q], S.sca(kb, SRHO)[a.lm_col[q]], acc);
    const float gr = 2.0f * acc;
    S.sca(kb, SGR)[j] = gr;
    float zd[D], gzd[D], gh[D];
    ld(S.arr(kb, ZD) + j * D, zd);
#pragma unroll
    for (int u = 0; u < D; ++u) gzd[u] = zd[u] > 0.0f ? w[O_DE + D * D + D + u] * gr : 0.0f;
    st(S.arr(kb, GZD) + j * D, gzd);
    ld(S.arr(kb, GH) + j * D, gh);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float acc2 = gh[i];
#pragma unroll
        for (int u = 0; u < D; ++u) acc2 = fmaf(w[O_DE + u * D + i], gzd[u], acc2);
        gh[i] = acc2;
    }
    float gps[D], zp[D], gz[D];
#pragma unroll
    for (int o = 0; o < D; ++o) gps[o] = a.alpha * gh[o];
    st(S.arr(kb, GPS) + j * D, gps);
    ld(S.arr(kb, ZP) + j * D, zp);
#pragma unroll
    for (int u = 0; u < D; ++u) {
        float acc2 = 0.0f;
#pragma unroll
        for (int o = 0; o < D; ++o) acc2 = fmaf(w[O_PS + D * F_PSI + D + o * D + u], gps[o], acc2);
        gz[u] = zp[u] > 0.0f ? acc2 : 0.0f;
    }
    st(S.arr(kb, GZ) + j * D, gz);
    float gx[F_PSI];
#pragma unroll
    for (int i = 0; i < F_PSI; ++i) {
        float acc2 = 0.0f;
#pragma unroll
        for (int u = 0; u < D; ++u) acc2 = fmaf(w[O_PS + u * F_PSI + i], gz[u], acc2);
        gx[i] = acc2;
    }
    st(S.arr(kb, GFO) + j * D, gx + D + 1);
    st(S.arr(kb, GFI) + j * D, gx + 2 * D + 1);
    float gmo[D], gmi[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
        float ao = 0.0f, ai = 0.0f;
#pragma unroll
        for (int v = 0; v < D; ++v) {
            ao = fmaf(w[O_PO + D * F_PHI + D + v * D + u], gx[D + 1 + v], ao);
            ai = fmaf(w[O_PI + D * F_PHI + D + v * D + u], gx[2 * D + 1 + v], ai);
        }
        gmo[u] = ao;
        gmi[u] = ai;
    }
    st(S.arr(kb, GMO) + j * D, gmo);
    st(S.arr(kb, GMI) + j * D, gmi);
#pragma unroll
    for (int i = 0; i < D; ++i) gh[i] += gx[i];
    st(S.arr(kb, GHN) + j * D, gh);
}

// Back through the first message layers for node j: per receiver and per sender
// edge sums, one message direction at a time.
__device__ __noinline__ void edge_back_node(const TrainArgs& a, const Sample& S, const float* w, int64_t b, int j) {
    const int kb = a.kbar;
    float gh[D];
    ld(S.arr(kb, GHN) + j * D, gh);
#pragma unroll 1
    for (int dir = 0; dir < 2; ++dir) {
        const float* wd = w + (dir ? O_PI : O_PO);
        const float sx = dir ? -1.0f : 1.0f;
        const float* P = S.arr(kb, dir ? PI : PO);
        const float* Q = S.arr(kb, dir ? QI : QO);
        const float* GM = S.arr(kb, dir ? GMI : GMO);
        float p[D], gm[D], gr[D], nn[D], gx[D], gy[D];
        ld(P + j * D, p);
        ld(GM + j * D, gm);
#pragma unroll
        for (int u = 0; u < D; ++u) gr[u] = nn[u] = gx[u] = gy[u] = 0.0f;
        for (int t = a.edge_ptr[b + j]; t < a.edge_ptr[b + j + 1]; ++t) {
            const int l = a.edge_src[t];
            const Edge e = edge(a, b, j, l, t);
            const float* q = Q + l * D;
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const float g = pre(p[u], q[u], wd + u * F_PHI, sx, e.dx, e.dy, e.nd) > 0.0f ? gm[u] : 0.0f;
                gr[u] += g;
                nn[u] = fmaf(g, e.nd, nn[u]);
                gx[u] = fmaf(g, e.dx, gx[u]);
                gy[u] = fmaf(g, e.dy, gy[u]);
            }
        }
        st(S.arr(kb, dir ? GRI : GRO) + j * D, gr);
        st(S.arr(kb, dir ? NI : NO) + j * D, nn);
        st(S.arr(kb, dir ? DXI : DXO) + j * D, gx);
        st(S.arr(kb, dir ? DYI : DYO) + j * D, gy);
        // edges leaving j: j is the sender, r the receiver
        float q[D], gs[D];
        ld(Q + j * D, q);
#pragma unroll
        for (int u = 0; u < D; ++u) gs[u] = 0.0f;
        for (int o = a.oe_ptr[b + j]; o < a.oe_ptr[b + j + 1]; ++o) {
            const int r = a.oe_recv[o];
            const Edge e = edge(a, b, r, j, a.oe_edge[o]);
            const float* pr = P + r * D;
            const float* gmr = GM + r * D;
#pragma unroll
            for (int u = 0; u < D; ++u)
                gs[u] += pre(pr[u], q[u], wd + u * F_PHI, sx, e.dx, e.dy, e.nd) > 0.0f ? gmr[u] : 0.0f;
        }
        st(S.arr(kb, dir ? GSI : GSO) + j * D, gs);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            float acc = gh[i];
#pragma unroll
            for (int u = 0; u < D; ++u) {
                acc = fmaf(wd[u * F_PHI + i], gr[u], acc);
                acc = fmaf(wd[u * F_PHI + D + i], gs[u], acc);
            }
            gh[i] = acc;
        }
    }
    st(S.arr(kb, GHN) + j * D, gh);
}

__global__ __launch_bounds__(TB) void train_grad_kernel(TrainArgs a) {
    __shared__ float w[TRAIN_NWB];
    __shared__ float tile[N_ROWS * CHP];
    __shared__ double red[TB / 64];
    const int s = a.s0 + blockIdx.x;
    const int sub = a.subs[s];
    const int64_t b = a.sub_ptr[sub];
    const int k = a.sub_ptr[sub + 1] - (int)b;
    const int kb = a.kbar;
    const Sample S{a.scratch + a.s_off[s], k};
    const float* cs = a.c + a.c_off[s];
    const int tid = threadIdx.x;
    auto load_w = [&](int blk) {
        __syncthreads();
        for (int i = tid; i < TRAIN_NWB; i += TB) w[i] = a.theta[(int64_t)blk * TRAIN_NWB + i];
        __syncthreads();
    };
    auto phase_pq = [&](int blk) {
        const float* H = S.hist(blk);
        for (int j = tid; j < k; j += TB) {
            float h[D], p[D], q[D];
            ld(H + j * D, h);
            pq(w + O_PO, h, p, q);
            st(S.arr(kb, PO) + j * D, p);
            st(S.arr(kb, QO) + j * D, q);
            pq(w + O_PI, h, p, q);
            st(S.arr(kb, PI) + j * D, p);
            st(S.arr(kb, QI) + j * D, q);
        }
        __syncthreads();
    };

    // Forward: H^0 = 0, then the kbar blocks.
    for (int64_t i = tid; i < (int64_t)k * D; i += TB) S.hist(0)[i] = 0.0f;
    for (int blk = 0; blk < kb; ++blk) {
        load_w(blk);
        phase_pq(blk);
        for (int j = tid; j < k; j += TB) block_node(a, S, w, S.hist(blk), S.hist(blk + 1), cs, b, j, false);
    }
    __syncthreads();
    for (int64_t i = tid; i < (int64_t)k * D; i += TB) S.arr(kb, GH)[i] = 0.0f;

    double sse = 0.0;
    for (int blk = kb - 1; blk >= 0; --blk) {
        load_w(blk);
        phase_pq(blk);
        const float* Hc = S.hist(blk + 1);
        // Block intermediates and the decoder of H^k.
        for (int j = tid; j < k; j += TB) {
            block_node(a, S, w, S.hist(blk), nullptr, cs, b, j, true);
            float h[D], zd[D], ud[D];
            ld(Hc + j * D, h);
            float r = w[O_DE + D * D + D + D];
#pragma unroll
            for (int u = 0; u < D; ++u) {
                float acc = w[O_DE + D * D + u];
#pragma unroll
                for (int i = 0; i < D; ++i) acc = fmaf(w[O_DE + u * D + i], h[i], acc);
                zd[u] = acc;
                ud[u] = fmaxf(acc, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < D; ++u) r = fmaf(w[O_DE + D * D + D + u], ud[u], r);
            st(S.arr(kb, ZD) + j * D, zd);
            st(S.arr(kb, UD) + j * D, ud);
            S.sca(kb, SR)[j] = r;
        }
        __syncthreads();
        // Residual of the local system.
        for (int j = tid; j < k; j += TB) {
            float acc = 0.0f;
            for (int q = a.lm_ptr[b + j]; q < a.lm_ptr[b + j + 1]; ++q)
                acc = fmaf(a.lm_val[q], S.sca(kb, SR)[a.lm_col[q]], acc);
            const float rho = acc - cs[j];
            S.sca(kb, SRHO)[j] = rho;
            sse += (double)rho * (double)rho;
        }
        __syncthreads();
        // Back through the decoder, Psi and the second message layers.
        for (int j = tid; j < k; j += TB) psi_back_node(a, S, w, cs, b, j);
        __syncthreads();
        // Back through the first message layers.
        for (int j = tid; j < k; j += TB) edge_back_node(a, S, w, b, j);
        __syncthreads();
        // The block's weight gradient; the gradient w.r.t. H^{k-1} becomes the carried one.
        float* gout = a.gpart + (int64_t)s * kb * TRAIN_NWB + (int64_t)blk * TRAIN_NWB;
        block_grad(a, S, cs, b, blk, tile, gout);
        for (int64_t i = tid; i < (int64_t)k * D; i += TB) S.arr(kb, GH)[i] = S.arr(kb, GHN)[i];
    }
    const double tot = block_sum_d(sse, red);
    if (tid == 0) a.sse[s] = tot;
}

// grad[e] = scale * sum_s gpart[s][e] in sample order.
__global__ void train_reduce_kernel(const float* gpart, int n, int64_t nth, double scale, float* grad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nth) return;
    double acc = 0.0;
    for (int s = 0; s < n; ++s) acc += (double)gpart[(int64_t)s * nth + e];
    grad[e] = (float)(scale * acc);
}

// Sum of squares of grad (one workgroup, fixed order) and of the samples' squared residuals.
__global__ __launch_bounds__(TB) void train_norm_kernel(const float* grad, int64_t nth, const double* sse, int n,
                                                       double* out) {
    __shared__ double red[TB / 64];
    double v = 0.0;
    for (int64_t e = threadIdx.x; e < nth; e += TB) v += (double)grad[e] * (double)grad[e];
    const double g2 = block_sum_d(v, red);
    if (threadIdx.x == 0) {
        double l = 0.0;
        for (int s = 0; s < n; ++s) l += sse[s];
        out[0] = g2;
        out[1] = l;
    }
}

__global__ void adam_kernel(float* theta, const float* grad, float* m, float* v, int64_t n, float gscale, float lr,
                            float b1, float b2, float bc1, float bc2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i] * gscale;
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// r = b - A u into r (FP64), one row per thread.
__global__ void train_resid_kernel(const int32_t* rowptr, const int32_t* col, const double* val, const double* bb,
                                   const double* u, double* r, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) acc = fma(val[q], u[col[q]], acc);
    r[i] = bb[i] - acc;
}

// c_i = R_i r / |R_i r| per sub-mesh (0 where R_i r = 0), in slot order.
__global__ __launch_bounds__(TB) void train_rhs_kernel(const int32_t* sub_ptr, const int32_t* sub_nodes,
                                                       const double* r, float* c) {
    __shared__ double red[TB / 64];
    __shared__ double inv;
    const int sub = blockIdx.x;
    const int b = sub_ptr[sub], k = sub_ptr[sub + 1] - b;
    double v = 0.0;
    for (int j = threadIdx.x; j < k; j += TB) {
        const double x = r[sub_nodes[b + j]];
        v = fma(x, x, v);
    }
    const double ss = block_sum_d(v, red);
    if (threadIdx.x == 0) inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += TB) c[b + j] = (float)(r[sub_nodes[b + j]] * inv);
}

}  // namespace

hipError_t launch_train_grad(const TrainArgs& a, int n, hipStream_t s) {
    hipLaunchKernelGGL(train_grad_kernel, dim3(n), dim3(TB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_train_reduce(const float* gpart, int n, int64_t nth, double scale, float* grad, double* out2,
                               const double* sse, hipStream_t s) {
    hipLaunchKernelGGL(train_reduce_kernel, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, s, gpart, n, nth, scale,
                       grad);
    hipLaunchKernelGGL(train_norm_kernel, dim3(1), dim3(TB), 0, s, grad, nth, sse, n, out2);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int64_t n, float gscale, float lr,
                       float b1, float b2, float bc1, float bc2, float eps, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, grad, m, v, n, gscale,
                       lr, b1, b2, bc1, bc2, eps);
    return hipGetLastError();
}

hipError_t launch_train_rhs(const int32_t* rowptr, const int32_t* col, const double* val, const double* bb,
                            const double* u, double* r, int n, const int32_t* sub_ptr, const int32_t* sub_nodes,
                            int K, float* c, hipStream_t s) {
    hipLaunchKernelGGL(train_resid_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rowptr, col, val, bb,
                       u, r, n);
    hipLaunchKernelGGL(train_rhs_kernel, dim3((unsigned)K), dim3(TB), 0, s, sub_ptr, sub_nodes, r, c);
    return hipGetLastError();
}

}  // namespace ddmgnn
