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

// sum_{j<k} f(j) as four interleaved partial sums (j mod 4), combined in a fixed
// order: several loads stay in flight.
template <typename F>
__device__ inline float sum4(int k, F f) {
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    int j = 0;
    for (; j + 4 <= k; j += 4) {
        a0 += f(j);
        a1 += f(j + 1);
        a2 += f(j + 2);
        a3 += f(j + 3);
    }
    if (j < k) a0 += f(j);
    if (j + 1 < k) a1 += f(j + 1);
    if (j + 2 < k) a2 += f(j + 2);
    return (a0 + a1) + (a2 + a3);
}

// Gradient of block `blk`'s weight e: a sum over the nodes of a product of
// two per-node quantities (fixed order).
__device__ __noinline__ float grad_entry(const TrainArgs& a, const Sample& S, const float* cs, int64_t b, int blk, int e) {
    const int kb = a.kbar;
    const int k = (int)S.k;
    const float* Hp = S.hist(blk);      // H^{k-1}
    const float* Hc = S.hist(blk + 1);  // H^k
    const float* A = nullptr;
    const float* B = nullptr;
    int ca = 0, cb = 0, sb = D;
    float sign = 1.0f;
    bool deg = false;
    if (e < O_PS) {
        const bool out = e < O_PI;
        const int r = e - (out ? O_PO : O_PI);
        const float* GR = S.arr(kb, out ? GRO : GRI);
        if (r < D * F_PHI) {
            const int u = r / F_PHI, i = r % F_PHI;
            ca = u;
            if (i < D) { A = GR; B = Hp; cb = i; }
            else if (i < 2 * D) { A = S.arr(kb, out ? GSO : GSI); B = Hp; cb = i - D; }
            else if (i == 2 * D) { A = S.arr(kb, out ? DXO : DXI); sign = out ? 1.0f : -1.0f; }
            else if (i == 2 * D + 1) { A = S.arr(kb, out ? DYO : DYI); sign = out ? 1.0f : -1.0f; }
            else { A = S.arr(kb, out ? NO : NI); }
        } else if (r < D * F_PHI + D) {
            A = GR; ca = r - D * F_PHI;
        } else if (r < D * F_PHI + D + D * D) {
            const int q = r - D * F_PHI - D;
            A = S.arr(kb, out ? GFO : GFI); ca = q / D;
            B = S.arr(kb, out ? MO : MI); cb = q % D;
        } else {
            A = S.arr(kb, out ? GFO : GFI); ca = r - D * F_PHI - D - D * D;
            deg = true;
        }
    } else if (e < O_DE) {
        const int r = e - O_PS;
        if (r < D * F_PSI) {
            const int u = r / F_PSI, i = r % F_PSI;
            A = S.arr(kb, GZ); ca = u;
            if (i < D) { B = Hp; cb = i; }
            else if (i == D) { B = cs; sb = 1; }
            else if (i < 2 * D + 1) { B = S.arr(kb, FO); cb = i - D - 1; }
            else { B = S.arr(kb, FI); cb = i - 2 * D - 1; }
        } else if (r < D * F_PSI + D) {
            A = S.arr(kb, GZ); ca = r - D * F_PSI;
        } else if (r < D * F_PSI + D + D * D) {
            const int q = r - D * F_PSI - D;
            A = S.arr(kb, GPS); ca = q / D;
            B = S.arr(kb, UP); cb = q % D;
        } else {
            A = S.arr(kb, GPS); ca = r - D * F_PSI - D - D * D;
        }
    } else {
        const int r = e - O_DE;
        if (r < D * D) {
            A = S.arr(kb, GZD); ca = r / D; B = Hc; cb = r % D;
        } else if (r < D * D + D) {
            A = S.arr(kb, GZD); ca = r - D * D;
        } else {
            // output layer: the scalar gradient of r_hat (stride 1)
            const float* G = S.sca(kb, SGR);
            const float* U = r < D * D + 2 * D ? S.arr(kb, UD) : nullptr;
            const int cu = r - D * D - D;
            return U ? sum4(k, [&](int j) { return G[j] * U[j * D + cu]; }) : sum4(k, [&](int j) { return G[j]; });
        }
    }
    float acc;
    if (deg)
        acc = sum4(k, [&](int j) { return A[j * D + ca] * (float)(a.edge_ptr[b + j + 1] - a.edge_ptr[b + j]); });
    else if (B)
        acc = sum4(k, [&](int j) { return A[j * D + ca] * B[j * sb + cb]; });
    else
        acc = sum4(k, [&](int j) { return A[j * D + ca]; });
    return sign * acc;
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
    __shared__ double red[TB / 64];
    const int s = blockIdx.x;
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
        for (int e = tid; e < TRAIN_NWB; e += TB) gout[e] = grad_entry(a, S, cs, b, blk, e);
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
