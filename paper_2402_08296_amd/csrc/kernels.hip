// VALU kernels of the DDM-GNN apply and of the Krylov iteration, all table
// driven (one launch serves every problem of a batch).
//
// One preconditioner apply (Sec. III.A) is three launches:
//   DSS forward     one workgroup per sub-mesh, largest first. Restricts the
//                   residual (s_i = |R_i r|, y0_i = (R_0 r)_i, c_i = R_i r / s_i)
//                   and runs the kbar DSS_theta blocks (Sec. III.B); writes
//                   s_i r~_i per slot. This file holds the FP64/FP32 VALU
//                   form; dss_mfma.hip the BF16 matrix-core form.
//   coarse_kernel   y = (R_0 A R_0^T)^{-1} y0 as a GEMV with the inverse
//                   formed at setup (step 1).
//   prolong_kernel  z(n) = sum over the sub-meshes holding n of
//                   w_i(n) s_i r~_i(n) + D_i(n) y_i; z = 0 at Dirichlet nodes
//                   (step 3), fused with the Krylov dot products that need z.
// The Krylov iteration adds the direction update with the SpMV and its dots,
// and the solution update with the convergence test. Every reduction writes
// one partial sum per workgroup; a finalize kernel with one workgroup per
// problem sums them in workgroup order and advances the scalar recurrences
// (alpha, beta, the test) on the device, so the host only polls a flag.
#include <hip/hip_runtime.h>

#include "ddmgnn.h"
#include "device.h"
#include "setup.h"

namespace ddmgnn {

namespace {

// Offsets in one weight block of latent width W (Sec. III.B; Table II counts).
template <int W>
struct DssLayout {
    static constexpr int IN_PHI = 2 * W + 3;                  // (h_j, h_l, d, |d|)
    static constexpr int IN_PSI = 3 * W + 1;                  // (h_j, c_j, phi_out, phi_in)
    static constexpr int OFF_PO = 0;                          // Phi_out
    static constexpr int OFF_PI = OFF_PO + W * IN_PHI + W + W * W + W;
    static constexpr int OFF_PS = OFF_PI + W * IN_PHI + W + W * W + W;
    static constexpr int OFF_DE = OFF_PS + W * IN_PSI + W + W * W + W;
    static constexpr int BLOCK_W = OFF_DE + W * W + W + W + 1;  // 11 d^2 + 15 d + 1
};
static_assert(DssLayout<10>::BLOCK_W == 1251 && DssLayout<5>::BLOCK_W == 351 && DssLayout<20>::BLOCK_W == 4701,
              "weight block size");

// Which reduction a finalize launch completes.
enum FinStage { FIN_PROLONG, FIN_SPMV, FIN_UPDATE, FIN_INIT, FIN_RESID, FIN_GM_DOT1, FIN_GM_DOT2, FIN_GM_ROT,
                FIN_GM_RESTART };

// ------------------------------------------------------------------ reductions
// Deterministic: fixed shuffle tree inside a wave, fixed order across waves,
// fixed order across workgroups (the last workgroup of a problem sums its
// partials), so a problem's result does not depend on what else is in the launch.
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <int BLOCK>
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int i = 0; i < BLOCK / 64; ++i) acc += sh[i];
        sh[BLOCK / 64] = acc;
    }
    __syncthreads();
    return sh[BLOCK / 64];
}

// NV block sums at once (one barrier round for all of them); the totals are
// valid in every thread. sh holds NV * (BLOCK / 64) doubles.
template <int NV, int BLOCK>
__device__ inline void block_sum_n(double (&v)[NV], double* sh) {
    constexpr int W = BLOCK / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0)
        for (int i = 0; i < NV; ++i) sh[i * W + w] = v[i];
    __syncthreads();
    for (int i = 0; i < NV; ++i) {
        double acc = 0.0;
        for (int k = 0; k < W; ++k) acc += sh[i * W + k];
        v[i] = acc;
    }
    __syncthreads();
}

// The restriction sums of the VALU DSS kernel over DSS_VBLOCK virtual threads
// (node j belongs to virtual thread j % DSS_VBLOCK, which sums its nodes in
// ascending order): thread t of a BLOCK-thread workgroup carries the virtual
// threads t + q BLOCK, and every wave's shuffle tree and the final sum over the
// virtual waves run in the order of a DSS_VBLOCK-thread workgroup, so both
// workgroup sizes of the kernel give the same bits.
constexpr int DSS_VBLOCK = 1024;
template <int BLOCK>
__device__ inline double vblock_sum(const double (&v)[DSS_VBLOCK / BLOCK], double* sh) {
    constexpr int VT = DSS_VBLOCK / BLOCK;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < VT; ++q) {
        const double x = wave_sum(v[q]);
        if (lane == 0) sh[w + q * (BLOCK / 64)] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int i = 0; i < DSS_VBLOCK / 64; ++i) acc += sh[i];
        sh[DSS_VBLOCK / 64] = acc;
    }
    __syncthreads();
    return sh[DSS_VBLOCK / 64];
}

// Two-kernel reductions of the Krylov iteration: every workgroup of a large
// kernel stores its partial sums with plain stores (no fence, no shared
// counter), and a finalize kernel with one workgroup per problem sums them in
// a fixed order after the large kernel has ended (the kernel boundary makes
// the stores visible). The sums therefore do not depend on which workgroup
// finishes last, nor on the other problems of the launch.
template <int NV>
__device__ inline void put_partials(double (&v)[NV], double* partials, int lb) {
    __shared__ double sh[NV * (VEC_BLOCK / 64)];
    block_sum_n<NV, VEC_BLOCK>(v, sh);
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) partials[i * VEC_GRID + lb] = v[i];
}

template <int NV>
__device__ inline void sum_partials(const double* __restrict__ partials, int nb, double (&out)[NV]) {
    __shared__ double sh[NV * (VEC_BLOCK / 64)];
    for (int i = 0; i < NV; ++i) out[i] = 0.0;
    for (int b = threadIdx.x; b < nb; b += VEC_BLOCK)
        for (int i = 0; i < NV; ++i) out[i] += partials[i * VEC_GRID + b];
    block_sum_n<NV, VEC_BLOCK>(out, sh);
}

// Work item of a vector-kernel workgroup: its problem and local workgroup.
struct Seg {
    const DevProb* P;
    int lb;
};
__device__ inline Seg seg(const DevProb* __restrict__ tab, const int2* __restrict__ blk) {
    const int2 w = blk[blockIdx.x];
    return {tab + w.x, w.y};
}

// Row groups (VEC_BLOCK consecutive rows each) of local workgroup lb of a
// problem with nblk workgroups (a multiple of N_XCD, the problem's first
// workgroup on die 0): the workgroups one die runs take one contiguous slab of
// groups, g0, g0 + gs, ... < g1, so a die's rows, their matrix columns and the
// vectors one kernel writes and the next reads stay in that die's L2. Every
// vector kernel uses the same map.
struct Rows {
    int g0, g1, gs;
};
__device__ inline Rows rows_of(int lb, int nblk, int n) {
    const int G = (n + VEC_BLOCK - 1) / VEC_BLOCK;
    const int x = lb % N_XCD;
    return {(int)((int64_t)G * x / N_XCD) + lb / N_XCD, (int)((int64_t)G * (x + 1) / N_XCD), nblk / N_XCD};
}

// ------------------------------------------------------------------ DSS forward (VALU)
template <typename T>
struct DssArgs {
    const DevProb* tab;
    const int2* work;         // (problem, sub-mesh), largest sub-meshes first
    int kbar;
    T alpha;
    int apply;                // 1: restrict P.r and write s r~; 0: read P.c_in, write r~
};

__device__ inline float relu(float x) { return fmaxf(x, 0.0f); }
__device__ inline double relu(double x) { return fmax(x, 0.0); }

// HREG: the latent state h of the thread's nodes stays in registers across all
// kbar blocks (FP32). Otherwise it lives in a per-slot global buffer (FP64,
// whose register footprint would spill).
// theta is a separate __restrict__ parameter so the compiler can prove the
// weight loads uniform and unclobbered and read them through the scalar cache.
// QLDS: Q lives in LDS (compile-time, so its accesses are ds_* rather than flat).
// SEP: the coordinate part of the message first layer is split per node,
// W1_d d_jl = W1_d x_l - W1_d x_j, and added to the projections (P and Q then
// carry it), so an edge only adds w_|d| |d_jl|; coordinates are centred on the
// sub-mesh to keep the cancellation small. Used for FP32; the FP64 path
// evaluates W1_d d_jl per edge.
// BIG: a sub-mesh of any size (beyond the kMaxSubNodes the others hold): h, c and Q
// live in per-slot global buffers and the node loops run over as many
// rounds of DSS_BLOCK nodes as the sub-mesh needs; the arithmetic per node is
// the same as the register-resident form's.
template <typename T, int D, bool HREG, bool QLDS, bool BIG = false, int BLOCK = DSS_BLOCK>
__global__ __launch_bounds__(BLOCK) void dss_kernel(DssArgs<T> a, const T* __restrict__ theta) {
    static_assert(!BIG || (!HREG && !QLDS), "a sub-mesh of any size keeps h and Q in global memory");
    using L = DssLayout<D>;
    constexpr int IN_PHI = L::IN_PHI, IN_PSI = L::IN_PSI, BLOCK_W = L::BLOCK_W;
    constexpr int OFF_PO = L::OFF_PO, OFF_PI = L::OFF_PI, OFF_PS = L::OFF_PS, OFF_DE = L::OFF_DE;
    constexpr bool SEP = sizeof(T) == 4;
    constexpr int NPT = (kMaxSubNodes + BLOCK - 1) / BLOCK;  // nodes per thread
    constexpr int VT = DSS_VBLOCK / BLOCK;                   // virtual threads per thread
    static_assert(VT == 1 || VT == 2, "512- or 1024-thread workgroups");
    const int2 wi = a.work[blockIdx.x];
    const DevProb& P = a.tab[wi.x];
    if (P.st && P.st->done) return;
    extern __shared__ unsigned char dyn_smem[];
    __shared__ double red[DSS_VBLOCK / 64 + 1];
    const int sub = wi.y;
    const int base = P.sub_ptr[sub];
    const int k = P.sub_ptr[sub + 1] - base;
    const T* xy;
    T* qglobal;
    if constexpr (SEP) {
        xy = P.xyc32;
        qglobal = P.qg32;
    } else {
        xy = P.xy64;
        qglobal = P.qg64;
    }
    T* Q = QLDS ? reinterpret_cast<T*>(dyn_smem) : qglobal + (size_t)base * 2 * D;
    const int32_t* __restrict__ edge_ptr = P.edge_ptr;
    const uint16_t* __restrict__ edge_src = P.edge_src;
    const float* __restrict__ edge_nd = P.edge_nd;
    double* __restrict__ out = P.local;
    const int tid = threadIdx.x;
    // rounds of BLOCK nodes (a compile-time count unless BIG)
    const int NT = BIG ? (k + BLOCK - 1) / BLOCK : NPT;
    constexpr int UNR = BIG ? 1 : NPT;  // unroll count of the node rounds

    T c[BIG ? 1 : NPT];
    T* cg = nullptr;  // BIG: c per slot in global memory
    if constexpr (BIG) {
        if constexpr (SEP)
            cg = P.c32 + base;
        else
            cg = P.c64 + base;
    }
    double s = 1.0;
    if (a.apply) {
        const double* __restrict__ r = P.r;
        double ssv[VT], yyv[VT], rv[BIG ? 1 : NPT];
#pragma unroll
        for (int q = 0; q < VT; ++q) ssv[q] = yyv[q] = 0.0;
#pragma unroll UNR
        for (int t = 0; t < NT; ++t) {
            const int j = tid + t * BLOCK;  // virtual thread j % DSS_VBLOCK = tid + (t % VT) BLOCK
            double v = 0.0;
            if (j < k) {
                v = r[P.sub_nodes[base + j]];
                if (VT == 1 || (t & 1) == 0) {
                    ssv[0] = fma(v, v, ssv[0]);
                    yyv[0] = fma(P.weights[base + j], v, yyv[0]);
                } else {
                    ssv[VT - 1] = fma(v, v, ssv[VT - 1]);
                    yyv[VT - 1] = fma(P.weights[base + j], v, yyv[VT - 1]);
                }
            }
            if constexpr (!BIG) rv[t] = v;
        }
        const double ss = vblock_sum<BLOCK>(ssv, red);
        const double yy = vblock_sum<BLOCK>(yyv, red);
        s = sqrt(ss);
        if (tid == 0) {
            P.s[sub] = s;
            P.y0[sub] = yy;
        }
        if (s == 0.0) {  // R_i r = 0: the local term is 0
            for (int j = tid; j < k; j += BLOCK) out[base + j] = 0.0;
            return;
        }
        if constexpr (BIG) {
            for (int j = tid; j < k; j += BLOCK) cg[j] = (T)(r[P.sub_nodes[base + j]] / s);
        } else {
#pragma unroll
            for (int t = 0; t < NPT; ++t) c[t] = (T)(rv[t] / s);
        }
    } else if constexpr (BIG) {
        for (int j = tid; j < k; j += BLOCK) cg[j] = (T)P.c_in[base + j];
    } else {
#pragma unroll
        for (int t = 0; t < NPT; ++t) {
            const int j = tid + t * BLOCK;
            c[t] = j < k ? (T)P.c_in[base + j] : (T)0;
        }
    }

    T hreg[HREG ? NPT : 1][D];
#pragma unroll
    for (int t = 0; t < (HREG ? NPT : 1); ++t)
#pragma unroll
        for (int u = 0; u < D; ++u) hreg[t][u] = (T)0;
    T* hg = nullptr;
    if constexpr (!HREG) {
        if constexpr (SEP)
            hg = P.hg32 + (size_t)base * D;
        else
            hg = P.hg64 + (size_t)base * D;
        for (int j = tid; j < k; j += BLOCK)
#pragma unroll
            for (int u = 0; u < D; ++u) hg[j * D + u] = (T)0;
    }

    for (int step = 0; step < a.kbar; ++step) {
        const T* __restrict__ w = theta + (size_t)step * BLOCK_W;
        const T* Wo = w + OFF_PO;                 // Phi_out W1 [D][IN_PHI]
        const T* bo = Wo + D * IN_PHI;
        const T* Vo = bo + D;                     // Phi_out W2 [D][D]
        const T* co = Vo + D * D;
        const T* Wi = w + OFF_PI;
        const T* bi = Wi + D * IN_PHI;
        const T* Vi = bi + D;
        const T* ci = Vi + D * D;
        const T* Wp = w + OFF_PS;                 // Psi W1 [D][IN_PSI]
        const T* bp = Wp + D * IN_PSI;
        const T* Vp = bp + D;
        const T* cp = Vp + D * D;

        // Phase A: neighbour projections Q_out = W1_out[:, D:2D] h, Q_in likewise.
#pragma unroll UNR
        for (int t = 0; t < NT; ++t) {
            const int j = tid + t * BLOCK;
            if (j < k) {
                T h[D];
#pragma unroll
                for (int v = 0; v < D; ++v) h[v] = HREG ? hreg[HREG ? t : 0][v] : hg[j * D + v];
                const T xl = xy[2 * (base + j)], yl = xy[2 * (base + j) + 1];
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    T qo = (T)0, qi = (T)0;
                    if (SEP) {  // Q_out += W1_d x_l, Q_in -= W1_d x_l (d_lj = -d_jl)
                        qo = fma(Wo[u * IN_PHI + 2 * D], xl, fma(Wo[u * IN_PHI + 2 * D + 1], yl, qo));
                        qi = -fma(Wi[u * IN_PHI + 2 * D], xl, Wi[u * IN_PHI + 2 * D + 1] * yl);
                    }
#pragma unroll
                    for (int v = 0; v < D; ++v) {
                        qo = fma(Wo[u * IN_PHI + D + v], h[v], qo);
                        qi = fma(Wi[u * IN_PHI + D + v], h[v], qi);
                    }
                    Q[j * 2 * D + u] = qo;
                    Q[j * 2 * D + D + u] = qi;
                }
            }
        }
        __syncthreads();

        // Phase B: per receiver, message sums over in-edges, then the Psi update.
#pragma unroll UNR
        for (int t = 0; t < NT; ++t) {
            const int j = tid + t * BLOCK;
            if (j < k) {
                T h[D];
#pragma unroll
                for (int v = 0; v < D; ++v) h[v] = HREG ? hreg[HREG ? t : 0][v] : hg[j * D + v];
                T po[D], pi[D], so[D], si[D];
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    T ao = bo[u], ai = bi[u];
#pragma unroll
                    for (int v = 0; v < D; ++v) {
                        ao = fma(Wo[u * IN_PHI + v], h[v], ao);
                        ai = fma(Wi[u * IN_PHI + v], h[v], ai);
                    }
                    po[u] = ao;
                    pi[u] = ai;
                    so[u] = (T)0;
                    si[u] = (T)0;
                }
                const T xj = xy[2 * (base + j)], yj = xy[2 * (base + j) + 1];
                if (SEP) {
#pragma unroll
                    for (int u = 0; u < D; ++u) {
                        po[u] = po[u] - fma(Wo[u * IN_PHI + 2 * D], xj, Wo[u * IN_PHI + 2 * D + 1] * yj);
                        pi[u] = fma(Wi[u * IN_PHI + 2 * D], xj, fma(Wi[u * IN_PHI + 2 * D + 1], yj, pi[u]));
                    }
                }
                const int e0 = edge_ptr[base + j], e1 = edge_ptr[base + j + 1];
                // Threads in their edge sums issue ahead of those in the dense
                // layers (same arithmetic; c1 and c2 solves 4-7% faster).
                __builtin_amdgcn_s_setprio(1);
                if (SEP) {
                    // Chunks of 2 edges as straight-line code: both rows are read from
                    // LDS before the sums. An edge past e1 reads the node's own row
                    // (the edge arrays are padded) and is masked with a 0 weight.
                    for (int e = e0; e < e1; e += 2) {
                        const bool in1 = e + 1 < e1;
                        const int l0 = edge_src[e], l1 = in1 ? (int)edge_src[e + 1] : j;
                        const T n0 = (T)edge_nd[e], n1 = (T)edge_nd[e + 1];
                        const T m1 = in1 ? (T)1 : (T)0;
                        T q0[2 * D], q1[2 * D];
#pragma unroll
                        for (int u = 0; u < 2 * D; ++u) {
                            q0[u] = Q[l0 * 2 * D + u];
                            q1[u] = Q[l1 * 2 * D + u];
                        }
#pragma unroll
                        for (int u = 0; u < D; ++u) {
                            const T wo = Wo[u * IN_PHI + 2 * D + 2], wi = Wi[u * IN_PHI + 2 * D + 2];
                            so[u] += relu(fma(wo, n0, po[u] + q0[u]));
                            si[u] += relu(fma(wi, n0, pi[u] + q0[D + u]));
                            so[u] = fma(m1, relu(fma(wo, n1, po[u] + q1[u])), so[u]);
                            si[u] = fma(m1, relu(fma(wi, n1, pi[u] + q1[D + u])), si[u]);
                        }
                    }
                } else {
                    for (int e = e0; e < e1; ++e) {
                        const int l = edge_src[e];
                        const T dx = xy[2 * (base + l)] - xj, dy = xy[2 * (base + l) + 1] - yj;
                        const T nr = sqrt(dx * dx + dy * dy);
                        const T* ql = Q + l * 2 * D;
#pragma unroll
                        for (int u = 0; u < D; ++u) {
                            T vo = po[u] + ql[u];
                            vo = fma(Wo[u * IN_PHI + 2 * D], dx, vo);
                            vo = fma(Wo[u * IN_PHI + 2 * D + 1], dy, vo);
                            vo = fma(Wo[u * IN_PHI + 2 * D + 2], nr, vo);
                            so[u] += relu(vo);
                            T vi = pi[u] + ql[D + u];
                            vi = fma(Wi[u * IN_PHI + 2 * D], -dx, vi);
                            vi = fma(Wi[u * IN_PHI + 2 * D + 1], -dy, vi);
                            vi = fma(Wi[u * IN_PHI + 2 * D + 2], nr, vi);
                            si[u] += relu(vi);
                        }
                    }
                }
                __builtin_amdgcn_s_setprio(0);
                const T deg = (T)(e1 - e0);
                T phio[D], phii[D];
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    T ao = co[u] * deg, ai = ci[u] * deg;
#pragma unroll
                    for (int v = 0; v < D; ++v) {
                        ao = fma(Vo[u * D + v], so[v], ao);
                        ai = fma(Vi[u * D + v], si[v], ai);
                    }
                    phio[u] = ao;
                    phii[u] = ai;
                }
                T hid[D];
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    T acc = bp[u];
#pragma unroll
                    for (int v = 0; v < D; ++v) acc = fma(Wp[u * IN_PSI + v], h[v], acc);
                    acc = fma(Wp[u * IN_PSI + D], BIG ? cg[j] : c[BIG ? 0 : t], acc);
#pragma unroll
                    for (int v = 0; v < D; ++v) acc = fma(Wp[u * IN_PSI + D + 1 + v], phio[v], acc);
#pragma unroll
                    for (int v = 0; v < D; ++v) acc = fma(Wp[u * IN_PSI + 2 * D + 1 + v], phii[v], acc);
                    hid[u] = relu(acc);
                }
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    T acc = cp[u];
#pragma unroll
                    for (int v = 0; v < D; ++v) acc = fma(Vp[u * D + v], hid[v], acc);
                    const T hn = fma(a.alpha, acc, h[u]);
                    if (HREG)
                        hreg[HREG ? t : 0][u] = hn;
                    else
                        hg[j * D + u] = hn;
                }
            }
        }
        __syncthreads();
    }

    // Decoder of the last block: r~_j = D^kbar(h_j).
    const T* dw = theta + (size_t)(a.kbar - 1) * BLOCK_W + OFF_DE;
    const T* db = dw + D * D;
    const T* dv = db + D;
    const T* dc = dv + D;
#pragma unroll UNR
    for (int t = 0; t < NT; ++t) {
        const int j = tid + t * BLOCK;
        if (j < k) {
            T h[D];
#pragma unroll
            for (int v = 0; v < D; ++v) h[v] = HREG ? hreg[HREG ? t : 0][v] : hg[j * D + v];
            T acc = dc[0];
#pragma unroll
            for (int u = 0; u < D; ++u) {
                T hu = db[u];
#pragma unroll
                for (int v = 0; v < D; ++v) hu = fma(dw[u * D + v], h[v], hu);
                acc = fma(dv[u], relu(hu), acc);
            }
            out[base + j] = a.apply ? s * (double)acc : (double)acc;
        }
    }
}

// ------------------------------------------------------------------ exact local solves
// DDM-LU (the paper's comparator, eq. (7)): local = (R_i A R_i^T)^{-1} R_i r with
// the inverse M formed at setup; one workgroup per sub-mesh, R_i r staged in
// LDS. M is symmetric, so local_j = sum_c M[c][j] x_c: a wavefront owns a
// strip of LU_STRIP columns (two per lane, 16-byte loads of contiguous row
// segments) and walks the rows in order with per-lane accumulators. Small
// sub-meshes (fewer strips than wavefronts) also split the rows into parts
// whose sums are added in part order through LDS. Also writes s_i = |R_i r|
// and y0_i = (R_0 r)_i like the DSS kernels.
constexpr int LU_STRIP = 128;
constexpr int LU_WAVES = DSS_BLOCK / 64;

__global__ __launch_bounds__(DSS_BLOCK) void lu_local_kernel(const DevProb* __restrict__ tab,
                                                            const int2* __restrict__ work) {
    const int2 wi = work[blockIdx.x];
    const DevProb& P = tab[wi.x];
    if (P.st && P.st->done) return;
    extern __shared__ double xs[];  // R_i r (k values; the launch reserves the work list's largest k)
    __shared__ double yp[LU_WAVES * LU_STRIP];  // parts * k <= LU_WAVES * LU_STRIP
    __shared__ double red[DSS_BLOCK / 64 + 1];
    const int sub = wi.y;
    const int base = P.sub_ptr[sub];
    const int k = P.sub_ptr[sub + 1] - base;
    const double* __restrict__ r = P.r;
    double ss = 0.0, yy = 0.0;
    for (int j = threadIdx.x; j < k; j += DSS_BLOCK) {
        const double v = r[P.sub_nodes[base + j]];
        xs[j] = v;
        ss = fma(v, v, ss);
        yy = fma(P.weights[base + j], v, yy);
    }
    // the barriers inside block_sum also publish xs
    ss = block_sum<DSS_BLOCK>(ss, red);
    yy = block_sum<DSS_BLOCK>(yy, red);
    if (threadIdx.x == 0) {
        P.s[sub] = sqrt(ss);
        P.y0[sub] = yy;
    }
    const int ld = (k + 1) & ~1;
    const double* __restrict__ M = P.lu_inv + P.lu_off[sub];
    double* __restrict__ out = P.local + base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ns = (k + LU_STRIP - 1) / LU_STRIP;
    const int parts = ns > 0 ? max(1, LU_WAVES / ns) : 1;
    const int rpp = (k + parts - 1) / parts;
    for (int t = wave; t < ns * parts; t += LU_WAVES) {
        const int strip = t % ns, part = t / ns;
        const int j = strip * LU_STRIP + 2 * lane;
        if (j >= k) continue;
        const int c0 = part * rpp, c1 = min(k, c0 + rpp);
        // column j + 1 may be the zero pad of an odd k
        const double2* __restrict__ col = reinterpret_cast<const double2*>(M + j);
        const int ld2 = ld >> 1;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
        for (int c = c0; c < c1; ++c) {
            const double2 v = col[(size_t)c * ld2];
            const double xc = xs[c];
            a0 = fma(v.x, xc, a0);
            a1 = fma(v.y, xc, a1);
        }
        if (parts == 1) {
            out[j] = a0;
            if (j + 1 < k) out[j + 1] = a1;
        } else {
            yp[part * k + j] = a0;
            if (j + 1 < k) yp[part * k + j + 1] = a1;
        }
    }
    if (parts > 1) {  // uniform over the workgroup (depends on k only)
        __syncthreads();
        for (int j = threadIdx.x; j < k; j += DSS_BLOCK) {
            double acc = yp[j];
            for (int q = 1; q < parts; ++q) acc += yp[q * k + j];
            out[j] = acc;
        }
    }
}

// ------------------------------------------------------------------ coarse solve
// y = A0inv y0: one workgroup per row (work item = (problem, row)), its four
// wavefronts over interleaved column segments, combined in a fixed order.
__global__ __launch_bounds__(VEC_BLOCK) void coarse_kernel(const DevProb* __restrict__ tab,
                                                          const int2* __restrict__ rows) {
    const int2 w = rows[blockIdx.x];
    const DevProb& P = tab[w.x];
    if (P.st && P.st->done) return;
    __shared__ double sh[VEC_BLOCK / 64];
    const int row = w.y, K = P.K;
    const double* __restrict__ a = P.a0inv + (size_t)row * K;
    const double* __restrict__ y0 = P.y0;
    double acc = 0.0;
    for (int j = threadIdx.x; j < K; j += VEC_BLOCK) acc = fma(a[j], y0[j], acc);
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < VEC_BLOCK / 64; ++i) t += sh[i];
        P.y[row] = t;
    }
}

// ------------------------------------------------------------------ prolong + dots
// The per-row loops live in force-inlined bodies whose pointer parameters are
// __restrict__: the pointers come from the problem table, and the no-alias
// scopes the inliner attaches let loads of later rows move above the stores
// of earlier ones.

// z over rows i0, i0 + stride, ... with the dots of the mode (FCG: <z, q_k>;
// PCG: <r, z>).
template <int MODE>
__device__ __forceinline__ void prolong_rows(const int32_t* __restrict__ node_ptr,
                                             const int32_t* __restrict__ node_slots,
                                             const int32_t* __restrict__ slot_sub,
                                             const double* __restrict__ weights, const double* __restrict__ local,
                                             const double* __restrict__ y, const uint8_t* __restrict__ dirichlet,
                                             const double* __restrict__ r, double* __restrict__ z,
                                             const double* __restrict__ q0, const double* __restrict__ q1,
                                             const double* __restrict__ q2, const double* __restrict__ q3, int m,
                                             bool unweighted, Rows rg, int n, double (&dots)[MAX_M + 1]) {
    // U rows of the thread at a time: the gathers of their first PM memberships
    // (most nodes have one or two) are all issued before any row is summed, so
    // the node -> slot -> value chains of the rows overlap. Each row is summed,
    // and the dots accumulated, in the same order as one row at a time.
    constexpr int U = 4, PM = 2;
    for (int gb = rg.g0; gb < rg.g1; gb += U * rg.gs) {
        int row[U], qb[U], qe[U];
        double wv[U][PM], lv[U][PM], yv[U][PM];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int gi = gb + u * rg.gs;
            const int i = gi * VEC_BLOCK + threadIdx.x;
            row[u] = gi < rg.g1 && i < n ? i : -1;
            qb[u] = qe[u] = 0;
            if (row[u] >= 0 && !dirichlet[i]) {
                qb[u] = node_ptr[i];
                qe[u] = node_ptr[i + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < PM; ++t) {
                wv[u][t] = lv[u][t] = yv[u][t] = 0.0;
                if (qb[u] + t < qe[u]) {
                    const int slot = node_slots[qb[u] + t];
                    wv[u][t] = weights[slot];
                    lv[u][t] = local[slot];
                    if (y) yv[u][t] = y[slot_sub[slot]];
                }
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = row[u];
            if (i < 0) continue;
            double zn = 0.0;
#pragma unroll
            for (int t = 0; t < PM; ++t)
                if (qb[u] + t < qe[u]) {
                    zn = fma(unweighted ? 1.0 : wv[u][t], lv[u][t], zn);
                    if (y) zn = fma(wv[u][t], yv[u][t], zn);
                }
            for (int q = qb[u] + PM; q < qe[u]; ++q) {
                const int slot = node_slots[q];
                const double w = weights[slot];
                zn = fma(unweighted ? 1.0 : w, local[slot], zn);
                if (y) zn = fma(w, y[slot_sub[slot]], zn);
            }
            z[i] = zn;
            if (MODE == DDMGNN_FCG) {
                dots[0] = fma(zn, q0[i], dots[0]);
                if (m > 1) dots[1] = fma(zn, q1[i], dots[1]);
                if (m > 2) dots[2] = fma(zn, q2[i], dots[2]);
                if (m > 3) dots[3] = fma(zn, q3[i], dots[3]);
            } else if (MODE == DDMGNN_PCG) {
                dots[0] = fma(r[i], zn, dots[0]);
            }
        }
    }
}

__global__ __launch_bounds__(VEC_BLOCK) void prolong_kernel(const DevProb* __restrict__ tab,
                                                           const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    KState* st = P.st;
    if (st && st->done) return;
    const int mode = st ? ia.mode : -1;
    const int m = ia.m;
    const int it = st ? st->it : 0;
    const double* qk[MAX_M] = {nullptr, nullptr, nullptr, nullptr};
    if (mode == DDMGNN_FCG)
        for (int i = 0; i < MAX_M; ++i) qk[i] = i < m ? P.q[ring_prev(it, m, i)] : nullptr;
    const double* y = ia.coarse ? P.y : nullptr;
    double dots[MAX_M + 1];
    for (int i = 0; i <= MAX_M; ++i) dots[i] = 0.0;
    const Rows rg = rows_of(g.lb, P.nblk, P.n);
    const bool uw = ia.unweighted;
    if (mode == DDMGNN_FGMRES) {  // z_j = M(v_j) goes to column j of Z, no dots
        prolong_rows<-1>(P.node_ptr, P.node_slots, P.slot_sub, P.weights, P.local, y, P.dirichlet, P.r,
                         P.gm_z + (size_t)st->gm_j * P.n, nullptr, nullptr, nullptr, nullptr, m, uw, rg, P.n, dots);
        return;
    }
    if (mode == DDMGNN_FCG)
        prolong_rows<DDMGNN_FCG>(P.node_ptr, P.node_slots, P.slot_sub, P.weights, P.local, y, P.dirichlet, P.r,
                                 P.z, qk[0], qk[1], qk[2], qk[3], m, uw, rg, P.n, dots);
    else if (mode == DDMGNN_PCG)
        prolong_rows<DDMGNN_PCG>(P.node_ptr, P.node_slots, P.slot_sub, P.weights, P.local, y, P.dirichlet, P.r,
                                 P.z, nullptr, nullptr, nullptr, nullptr, m, uw, rg, P.n, dots);
    else
        prolong_rows<-1>(P.node_ptr, P.node_slots, P.slot_sub, P.weights, P.local, y, P.dirichlet, P.r, P.z,
                         nullptr, nullptr, nullptr, nullptr, m, uw, rg, P.n, dots);
    if (mode < 0) return;
    put_partials<MAX_M + 1>(dots, P.partials, g.lb);
}

// ------------------------------------------------------------------ Krylov kernels
// Direction source of the iteration: z = M(r), or r itself for CG (M = I).
__device__ inline const double* dir_src(const DevProb& P, int mode) { return mode == DDMGNN_CG ? P.r : P.z; }

// Step length from <p, A p> and <p, r> (FCG) or rho (PCG/CG, Algorithm 1).
__device__ inline void set_alpha(KState* st, const double (&tot)[2], int mode, int slot) {
    const double pq = tot[0];
    st->pq[slot] = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
        st->status = isfinite(pq) ? DDMGNN_E_BREAKDOWN : DDMGNN_E_NONFINITE;
        st->done = 1;
        st->alpha = 0.0;
        return;
    }
    st->alpha = (mode == DDMGNN_FCG ? tot[1] : st->rho) / pq;
}

__device__ __forceinline__ void pupdate_rows(const double* __restrict__ z, double* __restrict__ pn,
                                             const double* __restrict__ p0, const double* __restrict__ p1,
                                             const double* __restrict__ p2, const double* __restrict__ p3, double b0,
                                             double b1, double b2, double b3, int m, Rows rg, int n) {
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int i = gi * VEC_BLOCK + threadIdx.x;
        if (i >= n) continue;
        double p = fma(b0, p0[i], z[i]);
        if (m > 1) p = fma(b1, p1[i], p);
        if (m > 2) p = fma(b2, p2[i], p);
        if (m > 3) p = fma(b3, p3[i], p);
        pn[i] = p;
    }
}

// p_new = z + sum_k beta[k] p_(it-1-k)  (FCG with m_max > 1)
__global__ __launch_bounds__(VEC_BLOCK) void pupdate_kernel(const DevProb* __restrict__ tab,
                                                           const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const KState* st = P.st;
    if (st->done) return;
    const int it = st->it, m = ia.m;
    const double* pk[MAX_M] = {nullptr, nullptr, nullptr, nullptr};
    for (int i = 0; i < MAX_M; ++i)
        if (i < m) pk[i] = P.p[ring_prev(it, m, i)];
    pupdate_rows(dir_src(P, ia.mode), P.p[ring_cur(it, m)], pk[0], pk[1], pk[2], pk[3], st->beta[0], st->beta[1],
                 st->beta[2], st->beta[3], m, rows_of(g.lb, P.nblk, P.n), P.n);
}

// CSR SpMV in groups of VEC_BLOCK consecutive rows (the groups of rows_of). The group's nonzeros are contiguous in CSR:
// they are staged through LDS with coalesced loads (value, and the gathered
// x(col)), then thread t sums row r0 + t in CSR order with the same fused
// multiply-add chain as a row-per-thread loop. A group with more than
// SPMV_CHUNK nonzeros is read row by row from global memory instead.
constexpr int SPMV_CHUNK = 2048;

template <class XF, class RowF>
__device__ __forceinline__ void spmv_groups(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                            const double* __restrict__ val, int n, int lb, int nblk, XF xof,
                                            RowF row_done) {
    __shared__ double sv[SPMV_CHUNK], sx[SPMV_CHUNK];
    const int tid = threadIdx.x;
    const Rows rg = rows_of(lb, nblk, n);
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int r0 = gi * VEC_BLOCK;
        const int r1 = min(n, r0 + VEC_BLOCK);
        const int e0 = rowptr[r0], e1 = rowptr[r1];
        const int row = r0 + tid;
        double acc = 0.0;
        if (e1 - e0 <= SPMV_CHUNK) {  // uniform over the workgroup
            for (int e = e0 + tid; e < e1; e += VEC_BLOCK) {
                sv[e - e0] = val[e];
                sx[e - e0] = xof(col[e]);
            }
            __syncthreads();
            if (row < r1)
                for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) acc = fma(sv[e - e0], sx[e - e0], acc);
            __syncthreads();
        } else if (row < r1) {
            for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) acc = fma(val[e], xof(col[e]), acc);
        }
        if (row < r1) row_done(row, acc);
    }
}

// q = A p with the dots the step length needs.
__global__ __launch_bounds__(VEC_BLOCK) void spmv_dots_kernel(const DevProb* __restrict__ tab,
                                                             const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    KState* st = P.st;
    if (st->done) return;
    const int slot = ring_cur(st->it, ia.m);
    const double* __restrict__ p = P.p[slot];
    double* __restrict__ q = P.q[slot];
    const double* __restrict__ r = P.r;
    double d[2] = {0.0, 0.0};
    spmv_groups(P.rowptr, P.col, P.val, P.n, g.lb, P.nblk, [&](int c) { return p[c]; },
                [&](int i, double acc) {
                    q[i] = acc;
                    d[0] = fma(p[i], acc, d[0]);
                    d[1] = fma(p[i], r[i], d[1]);
                });
    put_partials<2>(d, P.partials, g.lb);
}

// One kept direction (FCG(1), PCG, CG): p_new = z + beta p_old is formed on the
// fly for every column, q = A p_new, with the dots of spmv_dots_kernel. Every
// row evaluates fma(beta, p_old, z) identically, so q is exactly A times the
// stored p_new.
__global__ __launch_bounds__(VEC_BLOCK) void spmv_p_dots_kernel(const DevProb* __restrict__ tab,
                                                               const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    KState* st = P.st;
    if (st->done) return;
    const int it = st->it;
    const int slot = ring_cur(it, 1);
    const double* __restrict__ z = dir_src(P, ia.mode);
    const double* __restrict__ p_old = P.p[ring_prev(it, 1, 0)];
    double* __restrict__ p_new = P.p[slot];
    double* __restrict__ q = P.q[slot];
    const double* __restrict__ r = P.r;
    const double beta = st->beta[0];
    double d[2] = {0.0, 0.0};
    spmv_groups(P.rowptr, P.col, P.val, P.n, g.lb, P.nblk, [&](int c) { return fma(beta, p_old[c], z[c]); },
                [&](int i, double acc) {
                    const double pi = fma(beta, p_old[i], z[i]);
                    p_new[i] = pi;
                    q[i] = acc;
                    d[0] = fma(pi, acc, d[0]);
                    d[1] = fma(pi, r[i], d[1]);
                });
    put_partials<2>(d, P.partials, g.lb);
}

__device__ __forceinline__ void update_rows(double* __restrict__ u, double* __restrict__ r,
                                            const double* __restrict__ p, const double* __restrict__ q, double alpha,
                                            Rows rg, int n, double (&d)[1]) {
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int i = gi * VEC_BLOCK + threadIdx.x;
        if (i >= n) continue;
        u[i] = fma(alpha, p[i], u[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        d[0] = fma(ri, ri, d[0]);
    }
}

// u += alpha p; r -= alpha q; convergence test on |r| / |r_0|.
__global__ __launch_bounds__(VEC_BLOCK) void update_kernel(const DevProb* __restrict__ tab,
                                                          const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    KState* st = P.st;
    if (st->done) return;
    const int slot = ring_cur(st->it, ia.m);
    double d[1] = {0.0};
    update_rows(P.u, P.r, P.p[slot], P.q[slot], st->alpha, rows_of(g.lb, P.nblk, P.n), P.n, d);
    put_partials<1>(d, P.partials, g.lb);
}

__device__ __forceinline__ void residual_rows(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                              const double* __restrict__ val, const double* __restrict__ b,
                                              const double* __restrict__ u, double* __restrict__ u_copy,
                                              double* __restrict__ r, Rows rg, int n, double (&d)[1]) {
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int i = gi * VEC_BLOCK + threadIdx.x;
        if (i >= n) continue;
        double acc = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(val[e], u[col[e]], acc);
        const double ri = b[i] - acc;
        if (u_copy) u_copy[i] = u[i];
        if (r) r[i] = ri;
        d[0] = fma(ri, ri, d[0]);
    }
}

// u = u0; r = b - A u0 with |r|^2; zero the direction ring; initialise the state.
__global__ __launch_bounds__(VEC_BLOCK) void init_kernel(const DevProb* __restrict__ tab,
                                                        const int2* __restrict__ blk) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const Rows rg = rows_of(g.lb, P.nblk, P.n);
    double d[1] = {0.0};
    residual_rows(P.rowptr, P.col, P.val, P.b, P.u0, P.u, P.r, rg, P.n, d);
    for (int k = 0; k <= MAX_M; ++k) {
        double* __restrict__ pk = P.p[k];
        double* __restrict__ qk = P.q[k];
        for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
            const int i = gi * VEC_BLOCK + threadIdx.x;
            if (i < P.n) {
                pk[i] = 0.0;
                qk[i] = 0.0;
            }
        }
    }
    put_partials<1>(d, P.partials, g.lb);
}

// |b - A u|^2 of each problem into its state.
__global__ __launch_bounds__(VEC_BLOCK) void resid_kernel(const DevProb* __restrict__ tab,
                                                         const int2* __restrict__ blk) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    double d[1] = {0.0};
    residual_rows(P.rowptr, P.col, P.val, P.b, P.u, nullptr, nullptr, rows_of(g.lb, P.nblk, P.n), P.n, d);
    put_partials<1>(d, P.partials, g.lb);
}

// ------------------------------------------------------------------ FGMRES
// Restarted flexible GMRES (Saad's right-preconditioned variant): per step j,
// v_j = w / h_{j,j-1} (or r / beta at the start of a cycle) into the basis and
// into r, the apply z_j = M(v_j) into column j of Z, w = A z_j, then classical
// Gram-Schmidt against v_0..v_j run twice (three passes over the basis: dots;
// update and second dots; update and |w|), the Givens rotations and the
// residual estimate in a finalize kernel. At the end of a cycle u += Z y, then
// r = b - A u and a restart. The small arrays of a problem (ia.m = R steps per
// cycle) hold H [(R + 1) x R, column-major], cs [R], sn [R], g [R + 1],
// y [R] and tmp [R + 1].
struct GmSmall {
    double *H, *cs, *sn, *g, *y, *tmp;
    int ld;
};
__device__ inline GmSmall gm_small(const DevProb& P, int R) {
    double* b = P.gm_small;
    GmSmall m;
    m.ld = R + 1;
    m.H = b;
    m.cs = b + (size_t)(R + 1) * R;
    m.sn = m.cs + R;
    m.g = m.sn + R;
    m.y = m.g + R + 1;
    m.tmp = m.y + R;
    return m;
}

// v_j into the basis and into r (the input of the apply).
__global__ __launch_bounds__(VEC_BLOCK) void fgm_next_kernel(const DevProb* __restrict__ tab,
                                                            const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const KState* st = P.st;
    if (st->done) return;
    const int j = st->gm_j;
    const size_t n = P.n;
    double* __restrict__ vj = P.gm_v + j * n;
    const double* src = j == 0 ? P.r : vj;
    const double d = j == 0 ? st->gm_beta : st->gm_hnext;
    double* __restrict__ r = P.r;
    const Rows rg = rows_of(g.lb, P.nblk, P.n);
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int i = gi * VEC_BLOCK + threadIdx.x;
        if (i >= P.n) continue;
        const double v = src[i] / d;
        vj[i] = v;
        r[i] = v;
    }
}

// w = A z_j into basis column j + 1.
__global__ __launch_bounds__(VEC_BLOCK) void fgm_spmv_kernel(const DevProb* __restrict__ tab,
                                                            const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const KState* st = P.st;
    if (st->done) return;
    const int j = st->gm_j;
    const double* __restrict__ zj = P.gm_z + (size_t)j * P.n;
    double* __restrict__ w = P.gm_v + (size_t)(j + 1) * P.n;
    spmv_groups(P.rowptr, P.col, P.val, P.n, g.lb, P.nblk, [&](int c) { return zj[c]; },
                [&](int i, double acc) { w[i] = acc; });
}

// Partial sums of <w, v_k>, k = 0..j, over this workgroup's rows, eight basis
// vectors per sweep, into gm_part[k][lb].
__device__ inline void gm_dots(const DevProb& P, const Rows& rg, int lb, int j, const double* __restrict__ w) {
    __shared__ double sh[8 * (VEC_BLOCK / 64)];
    const size_t n = P.n;
    for (int k0 = 0; k0 <= j; k0 += 8) {
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
            const int i = gi * VEC_BLOCK + threadIdx.x;
            if (i >= P.n) continue;
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (k0 + q <= j) acc[q] = fma(wi, P.gm_v[(k0 + q) * n + i], acc[q]);
        }
        block_sum_n<8, VEC_BLOCK>(acc, sh);
        if (threadIdx.x == 0)
            for (int q = 0; q < 8 && k0 + q <= j; ++q) P.gm_part[(size_t)(k0 + q) * VEC_GRID + lb] = acc[q];
    }
}

__global__ __launch_bounds__(VEC_BLOCK) void fgm_gram_kernel(const DevProb* __restrict__ tab,
                                                            const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const KState* st = P.st;
    if (st->done) return;
    const int j = st->gm_j;
    gm_dots(P, rows_of(g.lb, P.nblk, P.n), g.lb, j, P.gm_v + (size_t)(j + 1) * P.n);
}

// w -= sum_k h_k v_k with h = tmp (the preceding dots); then (FINAL = false) the
// dots of the new w for the second pass, or (FINAL = true) the partial |w|^2.
template <bool FINAL>
__global__ __launch_bounds__(VEC_BLOCK) void fgm_orth_kernel(const DevProb* __restrict__ tab,
                                                            const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const KState* st = P.st;
    if (st->done) return;
    const int j = st->gm_j;
    const size_t n = P.n;
    const double* __restrict__ h = gm_small(P, ia.m).tmp;
    double* __restrict__ w = P.gm_v + (j + 1) * n;
    const Rows rg = rows_of(g.lb, P.nblk, P.n);
    double d[1] = {0.0};
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int i = gi * VEC_BLOCK + threadIdx.x;
        if (i >= P.n) continue;
        double wi = w[i];
        for (int k = 0; k <= j; ++k) wi = fma(-h[k], P.gm_v[k * n + i], wi);
        w[i] = wi;
        d[0] = fma(wi, wi, d[0]);
    }
    if (FINAL) {
        put_partials<1>(d, P.gm_part, g.lb);
    } else {
        gm_dots(P, rg, g.lb, j, w);
    }
}

// End of a cycle: u += sum_{q < k} y_q z_q.
__global__ __launch_bounds__(VEC_BLOCK) void fgm_xupd_kernel(const DevProb* __restrict__ tab,
                                                            const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const KState* st = P.st;
    if (st->done || !st->gm_end) return;
    const int k = st->gm_k;
    const size_t n = P.n;
    const double* __restrict__ y = gm_small(P, ia.m).y;
    double* __restrict__ u = P.u;
    const Rows rg = rows_of(g.lb, P.nblk, P.n);
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int i = gi * VEC_BLOCK + threadIdx.x;
        if (i >= P.n) continue;
        double ui = u[i];
        for (int q = 0; q < k; ++q) ui = fma(y[q], P.gm_z[q * n + i], ui);
        u[i] = ui;
    }
}

// End of a cycle: r = b - A u with its partial |r|^2.
__global__ __launch_bounds__(VEC_BLOCK) void fgm_resid_kernel(const DevProb* __restrict__ tab,
                                                             const int2* __restrict__ blk, IterArgs ia) {
    const Seg g = seg(tab, blk);
    const DevProb& P = *g.P;
    const KState* st = P.st;
    if (st->done || !st->gm_end) return;
    double d[1] = {0.0};
    residual_rows(P.rowptr, P.col, P.val, P.b, P.u, nullptr, P.r, rows_of(g.lb, P.nblk, P.n), P.n, d);
    put_partials<1>(d, P.partials, g.lb);
}

// Sums of gm_part[k][*] for k = 0..j in fixed order, one wavefront per k.
__device__ inline void gm_sum_dots(const DevProb& P, int j, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = wave; k <= j; k += VEC_BLOCK / 64) {
        double acc = 0.0;
        for (int b = lane; b < P.nblk; b += 64) acc += P.gm_part[(size_t)k * VEC_GRID + b];
        acc = wave_sum(acc);
        if (lane == 0) out[k] = acc;
    }
}

// Scalar recurrences of one problem from the partial sums of the preceding
// large kernel; one workgroup per problem (list[blockIdx.x], or blockIdx.x).
__global__ __launch_bounds__(VEC_BLOCK) void finalize_kernel(const DevProb* __restrict__ tab,
                                                            const int* __restrict__ list, int stage, IterArgs ia) {
    const DevProb& P = tab[list ? list[blockIdx.x] : blockIdx.x];
    KState* st = P.st;
    const bool always = stage == FIN_INIT || stage == FIN_RESID;
    if (!always && st->done) return;
    const bool t0 = threadIdx.x == 0;
    if (stage == FIN_PROLONG) {
        double tot[MAX_M + 1];
        sum_partials<MAX_M + 1>(P.partials, P.nblk, tot);
        if (!t0) return;
        const int it = st->it, m = ia.m;
        if (ia.mode == DDMGNN_FCG) {
            // p_new = z - sum_k (<z, q_k> / <p_k, q_k>) p_k
            for (int i = 0; i < MAX_M; ++i) st->beta[i] = i < m ? -tot[i] / st->pq[ring_prev(it, m, i)] : 0.0;
        } else {
            // Algorithm 1: beta = rho_{i+1} / rho_i, p = z + beta p
            const double rho_new = tot[0];
            st->beta[0] = it == 0 ? 0.0 : rho_new / st->rho;
            st->rho = rho_new;
        }
    } else if (stage == FIN_SPMV) {
        double tot[2];
        sum_partials<2>(P.partials, P.nblk, tot);
        if (t0) set_alpha(st, tot, ia.mode, ring_cur(st->it, ia.m));
    } else if (stage == FIN_UPDATE) {
        double tot[1];
        sum_partials<1>(P.partials, P.nblk, tot);
        if (!t0) return;
        const double rr = tot[0];
        st->it += 1;
        if (!isfinite(rr)) {
            st->status = DDMGNN_E_NONFINITE;
            st->done = 1;
            return;
        }
        st->rel = sqrt(rr) / st->r0n;
        if (ia.mode == DDMGNN_CG) {  // M = I: rho = <r, r>, beta = rho_new / rho_old
            st->beta[0] = rr / st->rho;
            st->rho = rr;
        }
        if (st->rel <= st->rtol || st->it >= st->max_it) st->done = 1;
    } else if (stage == FIN_INIT) {
        double tot[1];
        sum_partials<1>(P.partials, P.nblk, tot);
        if (!t0) return;
        st->r0n = sqrt(tot[0]);
        st->rtol = P.rtol;
        st->rel = tot[0] == 0.0 ? 0.0 : 1.0;
        st->alpha = 0.0;
        for (int i = 0; i < MAX_M; ++i) st->beta[i] = 0.0;
        for (int i = 0; i <= MAX_M; ++i) st->pq[i] = 1.0;
        st->rho = tot[0];
        st->rr_true = 0.0;
        st->it = 0;
        st->max_it = P.max_it;
        st->gm_beta = st->r0n;
        st->gm_hnext = 0.0;
        st->gm_j = 0;
        st->gm_k = 0;
        st->gm_end = 0;
        st->gm_conv = 0;
        st->status = isfinite(tot[0]) ? 0 : DDMGNN_E_NONFINITE;
        st->done = (tot[0] == 0.0 || !isfinite(tot[0]) || P.max_it <= 0) ? 1 : 0;
    } else if (stage == FIN_GM_DOT1 || stage == FIN_GM_DOT2) {
        // h_k of the Gram pass into tmp; the second pass adds to column j of H
        const GmSmall m = gm_small(P, ia.m);
        const int j = st->gm_j;
        gm_sum_dots(P, j, m.tmp);
        __syncthreads();
        for (int k = threadIdx.x; k <= j; k += VEC_BLOCK) {
            double* hk = m.H + (size_t)j * m.ld + k;
            *hk = stage == FIN_GM_DOT1 ? m.tmp[k] : *hk + m.tmp[k];
        }
    } else if (stage == FIN_GM_ROT) {
        double tot[1];
        sum_partials<1>(P.gm_part, P.nblk, tot);
        if (!t0) return;
        const GmSmall m = gm_small(P, ia.m);
        const int j = st->gm_j, R = ia.m;
        double* Hj = m.H + (size_t)j * m.ld;
        const double hn = sqrt(tot[0]);
        if (j == 0) m.g[0] = st->gm_beta;
        // earlier rotations on column j, then the one that zeroes h_{j+1,j}
        for (int i = 0; i < j; ++i) {
            const double t = m.cs[i] * Hj[i] + m.sn[i] * Hj[i + 1];
            Hj[i + 1] = -m.sn[i] * Hj[i] + m.cs[i] * Hj[i + 1];
            Hj[i] = t;
        }
        const double dd = hypot(Hj[j], hn);
        m.cs[j] = Hj[j] / dd;
        m.sn[j] = hn / dd;
        Hj[j] = dd;
        Hj[j + 1] = 0.0;
        m.g[j + 1] = -m.sn[j] * m.g[j];
        m.g[j] = m.cs[j] * m.g[j];
        st->it += 1;
        const double rel = fabs(m.g[j + 1]) / st->r0n;
        if (!isfinite(rel) || !isfinite(dd)) {
            st->status = DDMGNN_E_NONFINITE;
            st->done = 1;
            return;
        }
        if (!(dd > 0.0)) {  // H_j singular: no update possible
            st->status = DDMGNN_E_BREAKDOWN;
            st->done = 1;
            return;
        }
        st->rel = rel;
        st->gm_conv = rel <= st->rtol || hn == 0.0;
        if (st->gm_conv || j + 1 == R || st->it >= st->max_it) {
            // y = H_k^{-1} g (upper triangular), k = j + 1
            const int k = j + 1;
            for (int i = k - 1; i >= 0; --i) {
                double acc = m.g[i];
                for (int c = i + 1; c < k; ++c) acc -= m.H[(size_t)c * m.ld + i] * m.y[c];
                m.y[i] = acc / m.H[(size_t)i * m.ld + i];
            }
            st->gm_k = k;
            st->gm_end = 1;
        } else {
            st->gm_j = j + 1;
            st->gm_hnext = hn;
        }
    } else if (stage == FIN_GM_RESTART) {
        if (!st->gm_end) return;
        double tot[1];
        sum_partials<1>(P.partials, P.nblk, tot);
        if (!t0) return;
        st->gm_end = 0;
        st->gm_j = 0;
        st->gm_beta = sqrt(tot[0]);
        if (!isfinite(tot[0])) {
            st->status = DDMGNN_E_NONFINITE;
            st->done = 1;
        } else if (st->gm_conv || st->it >= st->max_it || tot[0] == 0.0) {
            st->done = 1;
        }
    } else {  // FIN_RESID
        double tot[1];
        sum_partials<1>(P.partials, P.nblk, tot);
        if (t0) st->rr_true = tot[0];
    }
}

// Entry points outside the solve run the solver's own code: y = A x with the
// grouped CSR SpMV over nblk workgroups, and x.y with the two-kernel
// reduction (per-workgroup partials over the row groups of rows_of, then one
// workgroup sums them in workgroup order).
__global__ __launch_bounds__(VEC_BLOCK) void spmv_kernel(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, const double* __restrict__ x,
                                                        double* __restrict__ y, int n, int nblk) {
    spmv_groups(rowptr, col, val, n, blockIdx.x, nblk, [&](int c) { return x[c]; },
                [&](int i, double acc) { y[i] = acc; });
}

__global__ __launch_bounds__(VEC_BLOCK) void dot_part_kernel(const double* __restrict__ x,
                                                            const double* __restrict__ y, int n, int nblk,
                                                            double* __restrict__ partials) {
    double d[1] = {0.0};
    const Rows rg = rows_of(blockIdx.x, nblk, n);
    for (int gi = rg.g0; gi < rg.g1; gi += rg.gs) {
        const int i = gi * VEC_BLOCK + threadIdx.x;
        if (i < n) d[0] = fma(x[i], y[i], d[0]);
    }
    put_partials<1>(d, partials, blockIdx.x);
}

__global__ __launch_bounds__(VEC_BLOCK) void dot_fin_kernel(const double* __restrict__ partials, int nblk,
                                                           double* __restrict__ out) {
    double tot[1];
    sum_partials<1>(partials, nblk, tot);
    if (threadIdx.x == 0) *out = tot[0];
}

// Copies the Krylov state of every problem of a table to one array (one host poll per chunk).
__global__ __launch_bounds__(VEC_BLOCK) void gather_states_kernel(const DevProb* __restrict__ tab, int n,
                                                                 KState* __restrict__ out) {
    const int i = blockIdx.x * VEC_BLOCK + threadIdx.x;
    if (i < n) out[i] = *tab[i].st;
}

inline hipError_t done(bool check) { return check ? hipGetLastError() : hipSuccess; }

}  // namespace

// ------------------------------------------------------------------ launchers
namespace {
template <int W>
hipError_t prepare_dss_valu_w(int precision, size_t shmem) {
    const bool f64 = precision == DDMGNN_FP64;
    const void* fn = f64 ? (const void*)dss_kernel<double, W, false, true> : (const void*)dss_kernel<float, W, true, true>;
    const void* fw = f64 ? (const void*)dss_kernel<double, W, false, true, false, DSS_WIDE_BLOCK>
                         : (const void*)dss_kernel<float, W, true, true, false, DSS_WIDE_BLOCK>;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    return e != hipSuccess ? e : hipFuncSetAttribute(fw, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
}

template <typename T, int W, bool HREG, int BLOCK>
void launch_dss_valu_b(const DssArgs<T>& a, const T* theta, int n_work, bool qlds, size_t shmem, hipStream_t s) {
    if (qlds)
        hipLaunchKernelGGL((dss_kernel<T, W, HREG, true, false, BLOCK>), dim3(n_work), dim3(BLOCK), shmem, s, a,
                           theta);
    else
        hipLaunchKernelGGL((dss_kernel<T, W, HREG, false, false, BLOCK>), dim3(n_work), dim3(BLOCK), 0, s, a, theta);
}

// A launch of fewer sub-meshes than the device has compute units takes the
// 1024-thread form (d <= 10): each sub-mesh then has twice the wavefronts to
// hide its latency (both forms give the same bits).
template <int W>
void launch_dss_valu_w(const DevProb* tab, const int2* work, int n_work, int precision, bool qlds, int kbar,
                       double alpha, int apply, const float* theta32, const double* theta64, size_t shmem,
                       hipStream_t s) {
    const bool wide = n_work < N_CU && W <= 10;  // at d = 20 the 1024-thread form spills
    if (precision == DDMGNN_FP64) {
        const DssArgs<double> a{tab, work, kbar, alpha, apply};
        if (wide) launch_dss_valu_b<double, W, false, DSS_WIDE_BLOCK>(a, theta64, n_work, qlds, shmem, s);
        else launch_dss_valu_b<double, W, false, DSS_BLOCK>(a, theta64, n_work, qlds, shmem, s);
    } else {
        const DssArgs<float> a{tab, work, kbar, (float)alpha, apply};
        if (wide) launch_dss_valu_b<float, W, true, DSS_WIDE_BLOCK>(a, theta32, n_work, qlds, shmem, s);
        else launch_dss_valu_b<float, W, true, DSS_BLOCK>(a, theta32, n_work, qlds, shmem, s);
    }
}
}  // namespace

hipError_t prepare_dss_valu(int precision, int d, size_t shmem) {
    switch (d) {
        case 5: return prepare_dss_valu_w<5>(precision, shmem);
        case 10: return prepare_dss_valu_w<10>(precision, shmem);
        case 20: return prepare_dss_valu_w<20>(precision, shmem);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dss_valu(const DevProb* tab, const int2* work, int n_work, int precision, int d, bool qlds,
                           int kbar, double alpha, int apply, const float* theta32, const double* theta64,
                           size_t shmem, hipStream_t s, bool check) {
    if (n_work <= 0) return hipSuccess;
    switch (d) {
        case 5: launch_dss_valu_w<5>(tab, work, n_work, precision, qlds, kbar, alpha, apply, theta32, theta64,
                                     shmem, s); break;
        case 10: launch_dss_valu_w<10>(tab, work, n_work, precision, qlds, kbar, alpha, apply, theta32, theta64,
                                       shmem, s); break;
        case 20: launch_dss_valu_w<20>(tab, work, n_work, precision, qlds, kbar, alpha, apply, theta32, theta64,
                                       shmem, s); break;
        default: return hipErrorInvalidValue;
    }
    return done(check);
}

hipError_t launch_dss_big(const DevProb* tab, const int2* work, int n_work, int precision, int d, int kbar,
                          double alpha, int apply, const float* theta32, const double* theta64, hipStream_t s,
                          bool check) {
    if (n_work <= 0) return hipSuccess;
    const DssArgs<double> a64{tab, work, kbar, alpha, apply};
    const DssArgs<float> a32{tab, work, kbar, (float)alpha, apply};
    const bool f64 = precision == DDMGNN_FP64;
    switch (d) {
        case 5:
            if (f64) hipLaunchKernelGGL((dss_kernel<double, 5, false, false, true>), dim3(n_work), dim3(DSS_BLOCK), 0, s, a64, theta64);
            else hipLaunchKernelGGL((dss_kernel<float, 5, false, false, true>), dim3(n_work), dim3(DSS_BLOCK), 0, s, a32, theta32);
            break;
        case 10:
            if (f64) hipLaunchKernelGGL((dss_kernel<double, 10, false, false, true>), dim3(n_work), dim3(DSS_BLOCK), 0, s, a64, theta64);
            else hipLaunchKernelGGL((dss_kernel<float, 10, false, false, true>), dim3(n_work), dim3(DSS_BLOCK), 0, s, a32, theta32);
            break;
        case 20:
            if (f64) hipLaunchKernelGGL((dss_kernel<double, 20, false, false, true>), dim3(n_work), dim3(DSS_BLOCK), 0, s, a64, theta64);
            else hipLaunchKernelGGL((dss_kernel<float, 20, false, false, true>), dim3(n_work), dim3(DSS_BLOCK), 0, s, a32, theta32);
            break;
        default: return hipErrorInvalidValue;
    }
    return done(check);
}

hipError_t prepare_lu_local() {
    return hipFuncSetAttribute((const void*)lu_local_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kMaxSubNodesAny * sizeof(double)));
}

hipError_t launch_lu_local(const DevProb* tab, const int2* work, int n_work, int max_k, hipStream_t s, bool check) {
    if (n_work <= 0) return hipSuccess;
    hipLaunchKernelGGL(lu_local_kernel, dim3(n_work), dim3(DSS_BLOCK), (size_t)max_k * sizeof(double), s, tab, work);
    return done(check);
}

hipError_t launch_coarse(const DevProb* tab, const int2* rows, int n_rows, hipStream_t s, bool check) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(coarse_kernel, dim3(n_rows), dim3(VEC_BLOCK), 0, s, tab, rows);
    return done(check);
}

hipError_t launch_prolong(const DevProb* tab, const int2* blk, int n_blk, int n_prob, const IterArgs& it,
                          hipStream_t s, bool check) {
    hipLaunchKernelGGL(prolong_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    if (it.mode >= 0 && it.mode != DDMGNN_FGMRES)
        hipLaunchKernelGGL(finalize_kernel, dim3(n_prob), dim3(VEC_BLOCK), 0, s, tab, (const int*)nullptr,
                           (int)FIN_PROLONG, it);
    return done(check);
}

hipError_t launch_krylov(const DevProb* tab, const int2* blk, int n_blk, int n_prob, const IterArgs& it,
                         hipStream_t s, bool check) {
    const int* all = nullptr;
    if (it.m == 1) {
        hipLaunchKernelGGL(spmv_p_dots_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    } else {
        hipLaunchKernelGGL(pupdate_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
        hipLaunchKernelGGL(spmv_dots_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    }
    hipLaunchKernelGGL(finalize_kernel, dim3(n_prob), dim3(VEC_BLOCK), 0, s, tab, all, (int)FIN_SPMV, it);
    hipLaunchKernelGGL(update_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    hipLaunchKernelGGL(finalize_kernel, dim3(n_prob), dim3(VEC_BLOCK), 0, s, tab, all, (int)FIN_UPDATE, it);
    return done(check);
}

hipError_t launch_fgmres_next(const DevProb* tab, const int2* blk, int n_blk, const IterArgs& it, hipStream_t s,
                              bool check) {
    hipLaunchKernelGGL(fgm_next_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    return done(check);
}

hipError_t launch_fgmres_step(const DevProb* tab, const int2* blk, int n_blk, int n_prob, const IterArgs& it,
                              hipStream_t s, bool check) {
    const int* all = nullptr;
    hipLaunchKernelGGL(fgm_spmv_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    hipLaunchKernelGGL(fgm_gram_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    hipLaunchKernelGGL(finalize_kernel, dim3(n_prob), dim3(VEC_BLOCK), 0, s, tab, all, (int)FIN_GM_DOT1, it);
    hipLaunchKernelGGL(fgm_orth_kernel<false>, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    hipLaunchKernelGGL(finalize_kernel, dim3(n_prob), dim3(VEC_BLOCK), 0, s, tab, all, (int)FIN_GM_DOT2, it);
    hipLaunchKernelGGL(fgm_orth_kernel<true>, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    hipLaunchKernelGGL(finalize_kernel, dim3(n_prob), dim3(VEC_BLOCK), 0, s, tab, all, (int)FIN_GM_ROT, it);
    hipLaunchKernelGGL(fgm_xupd_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    hipLaunchKernelGGL(fgm_resid_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk, it);
    hipLaunchKernelGGL(finalize_kernel, dim3(n_prob), dim3(VEC_BLOCK), 0, s, tab, all, (int)FIN_GM_RESTART, it);
    return done(check);
}

hipError_t launch_init(const DevProb* tab, const int2* blk, int n_blk, const int* list, int n_list, hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk);
    hipLaunchKernelGGL(finalize_kernel, dim3(n_list), dim3(VEC_BLOCK), 0, s, tab, list, (int)FIN_INIT, IterArgs{});
    return hipGetLastError();
}

hipError_t launch_resid(const DevProb* tab, const int2* blk, int n_blk, const int* list, int n_list, hipStream_t s) {
    hipLaunchKernelGGL(resid_kernel, dim3(n_blk), dim3(VEC_BLOCK), 0, s, tab, blk);
    hipLaunchKernelGGL(finalize_kernel, dim3(n_list), dim3(VEC_BLOCK), 0, s, tab, list, (int)FIN_RESID, IterArgs{});
    return hipGetLastError();
}

hipError_t launch_gather_states(const DevProb* tab, int n, KState* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_states_kernel, dim3((n + VEC_BLOCK - 1) / VEC_BLOCK), dim3(VEC_BLOCK), 0, s, tab, n,
                       out);
    return hipGetLastError();
}

hipError_t launch_spmv(const int32_t* rowptr, const int32_t* col, const double* val, const double* x, double* y,
                       int n, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(spmv_kernel, dim3(nblk), dim3(VEC_BLOCK), 0, s, rowptr, col, val, x, y, n, nblk);
    return hipGetLastError();
}

hipError_t launch_dot(const double* x, const double* y, int n, double* partials, double* out, hipStream_t s,
                      bool check) {
    const int nblk = vec_blocks(n);
    hipLaunchKernelGGL(dot_part_kernel, dim3(nblk), dim3(VEC_BLOCK), 0, s, x, y, n, nblk, partials);
    hipLaunchKernelGGL(dot_fin_kernel, dim3(1), dim3(VEC_BLOCK), 0, s, partials, nblk, out);
    return done(check);
}

}  // namespace ddmgnn
