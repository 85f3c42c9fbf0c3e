// DDM-GNN preconditioned flexible CG on MI355X (gfx950): device kernels and
// the C ABI declared in include/ddmgnn.h.
//
// One preconditioner apply (Sec. III.A) is three launches:
//   dss_kernel      one workgroup per sub-mesh, largest first. Restricts the
//                   residual (s_i = |R_i r|, y0_i = (R_0 r)_i, c_i = R_i r / s_i)
//                   and runs the kbar DSS_theta blocks (Sec. III.B) with the
//                   latent state in registers and the neighbour projections of
//                   the current block in LDS; writes s_i * r~_i per slot.
//   coarse_kernel   y = (R_0 A R_0^T)^{-1} y0 as a GEMV with the inverse
//                   formed at setup (step 1).
//   prolong_kernel  z(n) = sum over the sub-meshes holding n of
//                   w_i(n) s_i r~_i(n) + D_i(n) y_i; z = 0 at Dirichlet nodes
//                   (step 3), fused with the Krylov dot products that need z.
// The Krylov iteration adds pupdate, spmv_dots and update kernels. All scalar
// recurrences (alpha, beta, the convergence test) are computed on the device
// by the last workgroup of the kernel that finishes a reduction, so the host
// only polls a flag every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "ddmgnn.h"
#include "dss_mfma.h"
#include "setup.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(DDMGNN_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

constexpr int D = 10;                              // latent width (Sec. IV.B)
constexpr int IN_PHI = 2 * D + 3;                  // (h_j, h_l, d, |d|)
constexpr int IN_PSI = 3 * D + 1;                  // (h_j, c_j, phi_out, phi_in)
constexpr int OFF_PO = 0;                          // Phi_out
constexpr int OFF_PI = OFF_PO + D * IN_PHI + D + D * D + D;
constexpr int OFF_PS = OFF_PI + D * IN_PHI + D + D * D + D;
constexpr int OFF_DE = OFF_PS + D * IN_PSI + D + D * D + D;
constexpr int BLOCK_W = OFF_DE + D * D + D + D + 1;  // 11 d^2 + 15 d + 1
static_assert(BLOCK_W == 1251, "weight block size");

constexpr int VEC_BLOCK = 256;   // threads of the vector kernels
constexpr int VEC_GRID = 2048;   // max workgroups of the vector kernels (partials per dot)
constexpr int MAX_M = 4;         // largest FCG truncation supported
constexpr int DSS_BLOCK = 512;
constexpr int DSS_NPT = (ddmgnn::kMaxSubNodes + DSS_BLOCK - 1) / DSS_BLOCK;
constexpr size_t LDS_LIMIT = 160 * 1024;

// Device-resident Krylov scalars.
struct KState {
    double r0n;            // |r_0|
    double rtol;
    double rel;            // |r_it| / |r_0|
    double alpha;
    double beta[MAX_M];    // p_new = z + sum_k beta[k] * p_k (ring order of the call)
    double pq[MAX_M + 1];  // <p, A p> of each ring slot
    double rho;            // PCG/CG: <r, z> of the current iteration
    int it;
    int done;
    int status;
    int max_it;            // the update kernel raises done once it reaches max_it
};

// ------------------------------------------------------------------ reductions
// Deterministic: fixed shuffle tree inside a wave, fixed order across waves,
// fixed order across workgroups (the last workgroup sums the partials).
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

__device__ inline double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums NV values over the grid. Returns true in the last workgroup to
// finish, where out[] holds the totals (valid in every thread of that block).
template <int NV, int BLOCK>
__device__ bool grid_sum(const double (&v)[NV], double* partials, unsigned* counter, double (&out)[NV],
                         double* sh) {
    __shared__ int is_last;
    double bs[NV];
    for (int i = 0; i < NV; ++i) bs[i] = block_sum<BLOCK>(v[i], sh);
    if (threadIdx.x == 0) {
        for (int i = 0; i < NV; ++i) partials[i * VEC_GRID + blockIdx.x] = bs[i];
        __threadfence();
        unsigned t = atomicAdd(counter, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    for (int i = 0; i < NV; ++i) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += BLOCK) acc += load_coherent(&partials[i * VEC_GRID + b]);
        out[i] = block_sum<BLOCK>(acc, sh);
    }
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

// ------------------------------------------------------------------ DSS forward
template <typename T>
struct DssArgs {
    const int32_t* sub_ptr;
    const int32_t* work_order;
    const int32_t* edge_ptr;
    const uint16_t* edge_src;
    const T* xy;              // per slot (x, y); centred on the sub-mesh when SEP
    const float* edge_nd;     // per edge |d_jl| (SEP); padded by 8 entries
    const T* theta;           // kbar blocks of BLOCK_W
    const int32_t* sub_nodes;
    const double* weights;
    const double* r;          // apply: global residual
    const double* c_in;       // forward hook: per-slot inputs
    double* out;              // per slot: s_i r~_i (apply) or r~_i (hook)
    double* s_out;            // [K]
    double* y0_out;           // [K]
    T* qglobal;               // Q storage when it does not fit LDS
    T* hglobal;               // latent state storage when it is not kept in registers
    const KState* st;         // done flag (may be null)
    int kbar;
    T alpha;
    int apply;
    int q_in_lds;
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
template <typename T, bool HREG, bool QLDS>
__global__ __launch_bounds__(DSS_BLOCK) void dss_kernel(DssArgs<T> a, const T* __restrict__ theta) {
    constexpr bool SEP = sizeof(T) == 4;
    if (a.st && a.st->done) return;
    extern __shared__ unsigned char dyn_smem[];
    __shared__ double red[DSS_BLOCK / 64 + 1];
    const int sub = a.work_order[blockIdx.x];
    const int base = a.sub_ptr[sub];
    const int k = a.sub_ptr[sub + 1] - base;
    T* Q = QLDS ? reinterpret_cast<T*>(dyn_smem) : a.qglobal + (size_t)base * 2 * D;
    const int tid = threadIdx.x;

    T c[DSS_NPT];
    double s = 1.0;
    if (a.apply) {
        double ss = 0.0, yy = 0.0, rv[DSS_NPT];
#pragma unroll
        for (int t = 0; t < DSS_NPT; ++t) {
            const int j = tid + t * DSS_BLOCK;
            rv[t] = 0.0;
            if (j < k) {
                rv[t] = a.r[a.sub_nodes[base + j]];
                ss = fma(rv[t], rv[t], ss);
                yy = fma(a.weights[base + j], rv[t], yy);
            }
        }
        ss = block_sum<DSS_BLOCK>(ss, red);
        yy = block_sum<DSS_BLOCK>(yy, red);
        s = sqrt(ss);
        if (tid == 0) {
            a.s_out[sub] = s;
            a.y0_out[sub] = yy;
        }
        if (s == 0.0) {  // R_i r = 0: the local term is 0
            for (int j = tid; j < k; j += DSS_BLOCK) a.out[base + j] = 0.0;
            return;
        }
#pragma unroll
        for (int t = 0; t < DSS_NPT; ++t) c[t] = (T)(rv[t] / s);
    } else {
#pragma unroll
        for (int t = 0; t < DSS_NPT; ++t) {
            const int j = tid + t * DSS_BLOCK;
            c[t] = j < k ? (T)a.c_in[base + j] : (T)0;
        }
    }

    T hreg[HREG ? DSS_NPT : 1][D];
#pragma unroll
    for (int t = 0; t < (HREG ? DSS_NPT : 1); ++t)
#pragma unroll
        for (int u = 0; u < D; ++u) hreg[t][u] = (T)0;
    T* hg = HREG ? nullptr : a.hglobal + (size_t)base * D;
    if (!HREG)
        for (int j = tid; j < k; j += DSS_BLOCK)
#pragma unroll
            for (int u = 0; u < D; ++u) hg[j * D + u] = (T)0;

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
#pragma unroll
        for (int t = 0; t < DSS_NPT; ++t) {
            const int j = tid + t * DSS_BLOCK;
            if (j < k) {
                T h[D];
#pragma unroll
                for (int v = 0; v < D; ++v) h[v] = HREG ? hreg[HREG ? t : 0][v] : hg[j * D + v];
                const T xl = a.xy[2 * (base + j)], yl = a.xy[2 * (base + j) + 1];
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
#pragma unroll
        for (int t = 0; t < DSS_NPT; ++t) {
            const int j = tid + t * DSS_BLOCK;
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
                const T xj = a.xy[2 * (base + j)], yj = a.xy[2 * (base + j) + 1];
                if (SEP) {
#pragma unroll
                    for (int u = 0; u < D; ++u) {
                        po[u] = po[u] - fma(Wo[u * IN_PHI + 2 * D], xj, Wo[u * IN_PHI + 2 * D + 1] * yj);
                        pi[u] = fma(Wi[u * IN_PHI + 2 * D], xj, fma(Wi[u * IN_PHI + 2 * D + 1], yj, pi[u]));
                    }
                }
                const int e0 = a.edge_ptr[base + j], e1 = a.edge_ptr[base + j + 1];
                if (SEP) {
                    // Chunks of 2 edges as straight-line code: both rows are read from
                    // LDS before the sums. An edge past e1 reads the node's own row
                    // (the edge arrays are padded) and is masked with a 0 weight.
                    for (int e = e0; e < e1; e += 2) {
                        const bool in1 = e + 1 < e1;
                        const int l0 = a.edge_src[e], l1 = in1 ? (int)a.edge_src[e + 1] : j;
                        const T n0 = (T)a.edge_nd[e], n1 = (T)a.edge_nd[e + 1];
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
                        const int l = a.edge_src[e];
                        const T dx = a.xy[2 * (base + l)] - xj, dy = a.xy[2 * (base + l) + 1] - yj;
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
                    acc = fma(Wp[u * IN_PSI + D], c[t], acc);
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
#pragma unroll
    for (int t = 0; t < DSS_NPT; ++t) {
        const int j = tid + t * DSS_BLOCK;
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
            a.out[base + j] = a.apply ? s * (double)acc : (double)acc;
        }
    }
}

// ------------------------------------------------------------------ coarse solve
// y = A0inv y0, one wavefront per row.
__global__ __launch_bounds__(VEC_BLOCK) void coarse_kernel(const double* __restrict__ a0inv,
                                                          const double* __restrict__ y0, double* __restrict__ y,
                                                          int K, const KState* st) {
    if (st && st->done) return;
    const int row = blockIdx.x * (VEC_BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= K) return;
    const double* a = a0inv + (size_t)row * K;
    double acc = 0.0;
    for (int j = lane; j < K; j += 64) acc = fma(a[j], y0[j], acc);
    acc = wave_sum(acc);
    if (lane == 0) y[row] = acc;
}

// ------------------------------------------------------------------ prolong + dots
struct ProlongArgs {
    const int32_t* node_ptr;
    const int32_t* node_slots;
    const int32_t* slot_sub;
    const double* weights;
    const double* local;      // per slot s_i r~_i
    const double* y;          // coarse solution (null: no coarse term)
    const uint8_t* dirichlet;
    const double* r;
    double* z;
    const double* q[MAX_M];   // FCG: stored A p_k of the previous directions
    int pslot[MAX_M];         // ring slot of each previous direction (indexes KState::pq)
    int m;                    // number of stored directions (FCG)
    int n;
    int unweighted;
    int mode;                 // DDMGNN_FCG / DDMGNN_PCG; <0: no Krylov scalars (bare apply)
    double* partials;
    unsigned* counter;
    KState* st;
};

__global__ __launch_bounds__(VEC_BLOCK) void prolong_kernel(ProlongArgs a) {
    if (a.st && a.st->done) return;
    __shared__ double sh[VEC_BLOCK / 64 + 1];
    double dots[MAX_M + 1];
    for (int i = 0; i <= MAX_M; ++i) dots[i] = 0.0;
    for (int n = blockIdx.x * VEC_BLOCK + threadIdx.x; n < a.n; n += gridDim.x * VEC_BLOCK) {
        double z = 0.0;
        if (!a.dirichlet[n]) {
            for (int q = a.node_ptr[n]; q < a.node_ptr[n + 1]; ++q) {
                const int slot = a.node_slots[q];
                const double w = a.weights[slot];
                z = fma(a.unweighted ? 1.0 : w, a.local[slot], z);
                if (a.y) z = fma(w, a.y[a.slot_sub[slot]], z);
            }
        }
        a.z[n] = z;
        if (a.mode == DDMGNN_FCG) {
            for (int i = 0; i < MAX_M; ++i)
                if (i < a.m) dots[i] = fma(z, a.q[i][n], dots[i]);
        } else if (a.mode == DDMGNN_PCG) {
            dots[0] = fma(a.r[n], z, dots[0]);
        }
    }
    if (a.mode < 0) return;
    double tot[MAX_M + 1];
    if (!grid_sum<MAX_M + 1, VEC_BLOCK>(dots, a.partials, a.counter, tot, sh)) return;
    if (threadIdx.x != 0) return;
    KState* st = a.st;
    if (a.mode == DDMGNN_FCG) {
        // p_new = z - sum_k (<z, q_k> / <p_k, q_k>) p_k
        for (int i = 0; i < MAX_M; ++i) st->beta[i] = i < a.m ? -tot[i] / st->pq[a.pslot[i]] : 0.0;
    } else {
        // Algorithm 1: beta = rho_{i+1} / rho_i, p = z + beta p
        const double rho_new = tot[0];
        st->beta[0] = st->it == 0 ? 0.0 : rho_new / st->rho;
        st->rho = rho_new;
    }
}

// p_new = z + sum_k beta[k] p_k
__global__ __launch_bounds__(VEC_BLOCK) void pupdate_kernel(const double* __restrict__ z, double* p_new,
                                                           const double* p0, const double* p1, const double* p2,
                                                           const double* p3, int m, int n, const KState* st) {
    if (st->done) return;
    const double b0 = st->beta[0], b1 = st->beta[1], b2 = st->beta[2], b3 = st->beta[3];
    for (int i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        double p = z[i];
        if (m > 0) p = fma(b0, p0[i], p);
        if (m > 1) p = fma(b1, p1[i], p);
        if (m > 2) p = fma(b2, p2[i], p);
        if (m > 3) p = fma(b3, p3[i], p);
        p_new[i] = p;
    }
}

// q = A p with the dots the step length needs.
__global__ __launch_bounds__(VEC_BLOCK) void spmv_dots_kernel(const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ col,
                                                             const double* __restrict__ val,
                                                             const double* __restrict__ p, double* __restrict__ q,
                                                             const double* __restrict__ r, int n, int mode,
                                                             int slot, double* partials, unsigned* counter,
                                                             KState* st) {
    if (st->done) return;
    __shared__ double sh[VEC_BLOCK / 64 + 1];
    double d[2] = {0.0, 0.0};
    for (int i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        double acc = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(val[e], p[col[e]], acc);
        q[i] = acc;
        d[0] = fma(p[i], acc, d[0]);
        d[1] = fma(p[i], r[i], d[1]);
    }
    double tot[2];
    if (!grid_sum<2, VEC_BLOCK>(d, partials, counter, tot, sh)) return;
    if (threadIdx.x != 0) return;
    const double pq = tot[0];
    st->pq[slot] = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
        st->status = isfinite(pq) ? DDMGNN_E_BREAKDOWN : DDMGNN_E_NONFINITE;
        st->done = 1;
        st->alpha = 0.0;
        return;
    }
    // FCG: alpha = <p, r> / <p, A p>; PCG and CG (Algorithm 1): alpha = rho / <p, A p>
    st->alpha = (mode == DDMGNN_FCG ? tot[1] : st->rho) / pq;
}

// One truncation direction (FCG(1), PCG, CG): p_new = z + beta p_old is formed
// on the fly for every column, q = A p_new, with the dots of spmv_dots_kernel.
// Every row evaluates fma(beta, p_old, z) identically, so q is exactly A times
// the stored p_new.
__global__ __launch_bounds__(VEC_BLOCK) void spmv_p_dots_kernel(const int32_t* __restrict__ rowptr,
                                                               const int32_t* __restrict__ col,
                                                               const double* __restrict__ val,
                                                               const double* __restrict__ z,
                                                               const double* __restrict__ p_old,
                                                               double* __restrict__ p_new, double* __restrict__ q,
                                                               const double* __restrict__ r, int n, int mode, int slot,
                                                               double* partials, unsigned* counter, KState* st) {
    if (st->done) return;
    __shared__ double sh[VEC_BLOCK / 64 + 1];
    const double beta = st->beta[0];
    double d[2] = {0.0, 0.0};
    for (int i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        double acc = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int c = col[e];
            acc = fma(val[e], fma(beta, p_old[c], z[c]), acc);
        }
        const double pi = fma(beta, p_old[i], z[i]);
        p_new[i] = pi;
        q[i] = acc;
        d[0] = fma(pi, acc, d[0]);
        d[1] = fma(pi, r[i], d[1]);
    }
    double tot[2];
    if (!grid_sum<2, VEC_BLOCK>(d, partials, counter, tot, sh)) return;
    if (threadIdx.x != 0) return;
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

// u += alpha p; r -= alpha q; convergence test on |r| / |r_0|.
__global__ __launch_bounds__(VEC_BLOCK) void update_kernel(double* __restrict__ u, double* __restrict__ r,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ q, int n, int mode,
                                                          double* partials, unsigned* counter, KState* st) {
    if (st->done) return;
    __shared__ double sh[VEC_BLOCK / 64 + 1];
    const double alpha = st->alpha;
    double d[1] = {0.0};
    for (int i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        u[i] = fma(alpha, p[i], u[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        d[0] = fma(ri, ri, d[0]);
    }
    double tot[1];
    if (!grid_sum<1, VEC_BLOCK>(d, partials, counter, tot, sh)) return;
    if (threadIdx.x != 0) return;
    const double rr = tot[0];
    st->it += 1;
    if (!isfinite(rr)) {
        st->status = DDMGNN_E_NONFINITE;
        st->done = 1;
        return;
    }
    st->rel = sqrt(rr) / st->r0n;
    if (mode == DDMGNN_CG) {  // M = I: rho = <r, r>, beta = rho_new / rho_old
        st->beta[0] = rr / st->rho;
        st->rho = rr;
    }
    if (st->rel <= st->rtol || st->it >= st->max_it) st->done = 1;
}

// r = b - A u with |r|^2; zero the direction buffers; initialise the state.
__global__ __launch_bounds__(VEC_BLOCK) void init_kernel(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ b, const double* __restrict__ u,
                                                        double* __restrict__ r, double* const* ring, int n_ring,
                                                        int n, double rtol, int max_it, double* partials,
                                                        unsigned* counter, KState* st) {
    __shared__ double sh[VEC_BLOCK / 64 + 1];
    double d[1] = {0.0};
    for (int i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        double acc = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(val[e], u[col[e]], acc);
        const double ri = b[i] - acc;
        r[i] = ri;
        d[0] = fma(ri, ri, d[0]);
        for (int k = 0; k < n_ring; ++k) ring[k][i] = 0.0;
    }
    double tot[1];
    if (!grid_sum<1, VEC_BLOCK>(d, partials, counter, tot, sh)) return;
    if (threadIdx.x != 0) return;
    st->r0n = sqrt(tot[0]);
    st->rtol = rtol;
    st->rel = tot[0] == 0.0 ? 0.0 : 1.0;
    st->alpha = 0.0;
    for (int i = 0; i < MAX_M; ++i) st->beta[i] = 0.0;
    for (int i = 0; i <= MAX_M; ++i) st->pq[i] = 1.0;
    st->rho = tot[0];
    st->it = 0;
    st->max_it = max_it;
    st->status = isfinite(tot[0]) ? 0 : DDMGNN_E_NONFINITE;
    st->done = (tot[0] == 0.0 || !isfinite(tot[0]) || max_it <= 0) ? 1 : 0;
}

// Plain y = A x and a deterministic dot (hooks and the final true residual).
__global__ __launch_bounds__(VEC_BLOCK) void spmv_kernel(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, const double* __restrict__ x,
                                                        double* __restrict__ y, int n) {
    for (int i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        double acc = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(val[e], x[col[e]], acc);
        y[i] = acc;
    }
}

__global__ __launch_bounds__(VEC_BLOCK) void resid_kernel(const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val, const double* __restrict__ b,
                                                         const double* __restrict__ u, int n, double* partials,
                                                         unsigned* counter, double* out) {
    __shared__ double sh[VEC_BLOCK / 64 + 1];
    double d[1] = {0.0};
    for (int i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        double acc = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(val[e], u[col[e]], acc);
        const double ri = b[i] - acc;
        d[0] = fma(ri, ri, d[0]);
    }
    double tot[1];
    if (!grid_sum<1, VEC_BLOCK>(d, partials, counter, tot, sh)) return;
    if (threadIdx.x == 0) *out = tot[0];
}

__global__ __launch_bounds__(VEC_BLOCK) void dot_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                       int64_t n, double* partials, unsigned* counter,
                                                       double* out) {
    __shared__ double sh[VEC_BLOCK / 64 + 1];
    double d[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)VEC_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VEC_BLOCK)
        d[0] = fma(x[i], y[i], d[0]);
    double tot[1];
    if (!grid_sum<1, VEC_BLOCK>(d, partials, counter, tot, sh)) return;
    if (threadIdx.x == 0) *out = tot[0];
}

// ------------------------------------------------------------------ helpers
int vec_grid(int64_t n) {
    int64_t g = (n + VEC_BLOCK - 1) / VEC_BLOCK;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, VEC_GRID));
}

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = count;
        if (count == 0) return hipSuccess;
        return hipMalloc(&p, count * sizeof(T));
    }
    hipError_t upload(const T* src, size_t count, hipStream_t s) {
        hipError_t e = alloc(count);
        if (e != hipSuccess || count == 0) return e;
        e = hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }
};

}  // namespace

// ------------------------------------------------------------------ handles
struct ddmgnn_ctx {
    hipStream_t stream = nullptr;   // the caller's stream: all work runs here
    hipStream_t launch = nullptr;   // where kernels are enqueued (= stream, or cap while capturing)
    hipStream_t cap = nullptr;      // own non-blocking stream for graph capture (the null stream cannot be captured)
    int device = 0;
    DevBuf<double> partials;
    DevBuf<unsigned> counters;
    DevBuf<double> scalar;
    double* host_pinned = nullptr;
};

struct ddmgnn_model {
    int kbar = 0, d = 0;
    double alpha = 0;
    std::vector<float> theta;
    std::vector<ddmgnn::MfmaStep> mfma_steps;  // per block: A operands and lane constants
    std::vector<ddmgnn::MfmaDec> mfma_dec;
};

struct ddmgnn_problem {
    ddmgnn_ctx* ctx = nullptr;
    ddmgnn::HostSetup hs;
    int kbar = 0;
    double alpha = 0;
    // matrix and vectors
    DevBuf<int32_t> rowptr, col;
    DevBuf<double> val, b, u0;
    DevBuf<uint8_t> dirichlet;
    // decomposition
    DevBuf<int32_t> sub_ptr, sub_nodes, work_order, edge_ptr, node_ptr, node_slots, slot_sub;
    DevBuf<uint16_t> edge_src;
    DevBuf<double> weights, xy64, a0inv;
    DevBuf<float> xyc32;  // per slot, centred on the sub-mesh
    DevBuf<float> theta32;
    DevBuf<double> theta64;
    DevBuf<ddmgnn::MfmaStep> mfma_steps;
    DevBuf<ddmgnn::MfmaDec> mfma_dec;
    DevBuf<ddmgnn::TileNode> tiles;
    DevBuf<uint32_t> erec;   // padded by 8 entries
    bool mfma_fits = false;  // every sub-mesh fits the MFMA kernel's LDS
    DevBuf<float> edge_nd;
    // apply buffers
    DevBuf<double> s, y0, y, local;
    DevBuf<double> qglobal64, hglobal64;
    DevBuf<float> qglobal32;
    // Krylov state
    DevBuf<double> u, r, z;
    DevBuf<double> ring;  // (MAX_M + 1) p vectors then (MAX_M + 1) q vectors
    DevBuf<double*> ring_ptrs;
    DevBuf<KState> st;
    DevBuf<double> partials;
    DevBuf<unsigned> counters;
    // captured FCG chunk (kernels and pointers fixed per options key)
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_key = 0;
    ~ddmgnn_problem() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    }
};

namespace {

// Allocates the global fallback buffers a DSS launch of this precision needs
// (done before any stream capture, which must not allocate).
int prepare_dss(ddmgnn_problem* P, int precision) {
    const int64_t sk = P->hs.sk;
    if (precision == DDMGNN_BF16 && P->mfma_fits) {
        HIP_TRY(ddmgnn::prepare_dss_mfma(ddmgnn::MFMA_LDS_LIMIT));
        return DDMGNN_OK;
    }
    if (precision == DDMGNN_BF16) precision = DDMGNN_FP32;  // sub-mesh too large for the MFMA kernel
    const bool f64 = precision == DDMGNN_FP64;
    const size_t need = (size_t)P->hs.max_k * 2 * D * (f64 ? sizeof(double) : sizeof(float));
    const bool in_lds = need + 1024 <= LDS_LIMIT;
    if (!in_lds) {
        if (f64 && P->qglobal64.n == 0) HIP_TRY(P->qglobal64.alloc((size_t)sk * 2 * D));
        if (!f64 && P->qglobal32.n < (size_t)sk * 2 * D) HIP_TRY(P->qglobal32.alloc((size_t)sk * 2 * D));
    }
    if (f64 && P->hglobal64.n == 0) HIP_TRY(P->hglobal64.alloc((size_t)sk * D));
    if (in_lds) {
        const void* fn = f64 ? (const void*)dss_kernel<double, false, true> : (const void*)dss_kernel<float, true, true>;
        HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
    }
    return DDMGNN_OK;
}

// capturing: the stream is being captured into a graph; prepare_dss has run
// and no HIP call other than the launch is allowed.
int launch_dss(ddmgnn_problem* P, int precision, bool apply, const double* r, const double* c_in, double* out,
               const KState* st, bool capturing = false) {
    if (!capturing)
        if (int rc = prepare_dss(P, precision)) return rc;
    hipStream_t s = P->ctx->launch;
    const int K = P->hs.K;
    if (precision == DDMGNN_BF16 && P->mfma_fits) {
        ddmgnn::DssMfmaArgs a{};
        a.sub_ptr = P->sub_ptr.p; a.work_order = P->work_order.p; a.edge_ptr = P->edge_ptr.p;
        a.erec = P->erec.p; a.tiles = P->tiles.p;
        a.sub_nodes = P->sub_nodes.p; a.weights = P->weights.p; a.r = r; a.c_in = c_in; a.out = out;
        a.s_out = P->s.p; a.y0_out = P->y0.p; a.done = st ? &st->done : nullptr;
        a.steps = P->mfma_steps.p; a.dec = P->mfma_dec.p; a.kbar = P->kbar; a.alpha = (float)P->alpha;
        a.apply = apply;
        HIP_TRY(ddmgnn::launch_dss_mfma(a, K, ddmgnn::MFMA_LDS_LIMIT, s, !capturing));
        return DDMGNN_OK;
    }
    if (precision == DDMGNN_BF16) precision = DDMGNN_FP32;  // sub-mesh too large for the MFMA kernel
    const bool f64 = precision == DDMGNN_FP64;
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    const size_t need = (size_t)P->hs.max_k * 2 * D * esz;
    const bool in_lds = need + 1024 <= LDS_LIMIT;
    const size_t shmem = in_lds ? need : 0;
    if (f64) {
        DssArgs<double> a{};
        a.sub_ptr = P->sub_ptr.p; a.work_order = P->work_order.p; a.edge_ptr = P->edge_ptr.p;
        a.edge_src = P->edge_src.p; a.xy = P->xy64.p; a.theta = P->theta64.p; a.sub_nodes = P->sub_nodes.p;
        a.weights = P->weights.p; a.r = r; a.c_in = c_in; a.out = out; a.s_out = P->s.p; a.y0_out = P->y0.p;
        a.qglobal = P->qglobal64.p; a.hglobal = P->hglobal64.p; a.st = st; a.kbar = P->kbar; a.alpha = P->alpha;
        a.apply = apply; a.q_in_lds = in_lds;
        if (in_lds) {
            hipLaunchKernelGGL((dss_kernel<double, false, true>), dim3(K), dim3(DSS_BLOCK), shmem, s, a,
                               (const double*)P->theta64.p);
        } else {
            hipLaunchKernelGGL((dss_kernel<double, false, false>), dim3(K), dim3(DSS_BLOCK), 0, s, a,
                               (const double*)P->theta64.p);
        }
    } else {
        DssArgs<float> a{};
        a.sub_ptr = P->sub_ptr.p; a.work_order = P->work_order.p; a.edge_ptr = P->edge_ptr.p;
        a.edge_src = P->edge_src.p; a.xy = P->xyc32.p; a.edge_nd = P->edge_nd.p; a.theta = P->theta32.p;
        a.sub_nodes = P->sub_nodes.p;
        a.weights = P->weights.p; a.r = r; a.c_in = c_in; a.out = out; a.s_out = P->s.p; a.y0_out = P->y0.p;
        a.qglobal = P->qglobal32.p; a.hglobal = nullptr; a.st = st; a.kbar = P->kbar; a.alpha = (float)P->alpha;
        a.apply = apply; a.q_in_lds = in_lds;
        if (in_lds) {
            hipLaunchKernelGGL((dss_kernel<float, true, true>), dim3(K), dim3(DSS_BLOCK), shmem, s, a,
                               (const float*)P->theta32.p);
        } else {
            hipLaunchKernelGGL((dss_kernel<float, true, false>), dim3(K), dim3(DSS_BLOCK), 0, s, a,
                               (const float*)P->theta32.p);
        }
    }
    if (!capturing) HIP_TRY(hipGetLastError());
    return DDMGNN_OK;
}

// Enqueue one preconditioner apply z = M(r) with the Krylov dots of `mode`.
// ev (optional): events recorded after the DSS (ev[1]), coarse (ev[2]) and prolong (ev[3]) launches.
int enqueue_apply(ddmgnn_problem* P, const ddmgnn_solve_opts& o, const double* r, double* z, int mode,
                  double* const* qk, const int* pslot, int m, KState* st, hipEvent_t* ev = nullptr,
                  bool capturing = false) {
    int rc = launch_dss(P, o.precision, true, r, nullptr, P->local.p, st, capturing);
    if (rc) return rc;
    hipStream_t s = P->ctx->launch;
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    const int K = P->hs.K;
    if (o.coarse) {
        hipLaunchKernelGGL(coarse_kernel, dim3((K + 3) / 4), dim3(VEC_BLOCK), 0, s, P->a0inv.p, P->y0.p, P->y.p, K,
                           st);
    }
    if (ev) HIP_TRY(hipEventRecord(ev[2], s));
    ProlongArgs a{};
    a.node_ptr = P->node_ptr.p; a.node_slots = P->node_slots.p; a.slot_sub = P->slot_sub.p;
    a.weights = P->weights.p; a.local = P->local.p; a.y = o.coarse ? P->y.p : nullptr;
    a.dirichlet = P->dirichlet.p; a.r = r; a.z = z;
    for (int i = 0; i < MAX_M; ++i) {
        a.q[i] = (qk && i < m) ? qk[i] : nullptr;
        a.pslot[i] = (pslot && i < m) ? pslot[i] : 0;
    }
    a.m = m; a.n = (int)P->hs.n; a.unweighted = o.prolong == DDMGNN_PROLONG_UNWEIGHTED; a.mode = mode;
    a.partials = P->partials.p; a.counter = P->counters.p; a.st = st;
    hipLaunchKernelGGL(prolong_kernel, dim3(vec_grid(P->hs.n)), dim3(VEC_BLOCK), 0, s, a);
    if (!capturing) HIP_TRY(hipGetLastError());
    if (ev) HIP_TRY(hipEventRecord(ev[3], s));
    return DDMGNN_OK;
}

// Enqueue FCG/PCG/CG iteration `it` (ring slots depend on it % (m+1)). ev:
// optional 5 profiling events (before DSS, after DSS/coarse/prolong, end).
int enqueue_iteration(ddmgnn_problem* P, const ddmgnn_solve_opts& o, int it, hipEvent_t* ev,
                      bool capturing = false) {
    hipStream_t s = P->ctx->launch;
    const int64_t n = P->hs.n;
    const int grid = vec_grid(n);
    const int mode = o.krylov;
    const int m = mode == DDMGNN_FCG ? o.m_max : 1;
    const int nring = m + 1;
    const int cur = it % nring;
    double* pv_cur = P->ring.p + (size_t)cur * n;
    double* qv_cur = P->ring.p + (size_t)(MAX_M + 1 + cur) * n;
    double* prev_p[MAX_M] = {nullptr, nullptr, nullptr, nullptr};
    double* prev_q[MAX_M] = {nullptr, nullptr, nullptr, nullptr};
    int prev_slot[MAX_M] = {0, 0, 0, 0};
    for (int kk = 0; kk < m; ++kk) {
        const int sl = ((it - 1 - kk) % nring + nring) % nring;
        prev_p[kk] = P->ring.p + (size_t)sl * n;
        prev_q[kk] = P->ring.p + (size_t)(MAX_M + 1 + sl) * n;
        prev_slot[kk] = sl;
    }
    const double* zsrc = P->z.p;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    if (mode == DDMGNN_CG) {
        zsrc = P->r.p;
        if (ev)
            for (int q = 1; q < 4; ++q) HIP_TRY(hipEventRecord(ev[q], s));
    } else {
        int rc = enqueue_apply(P, o, P->r.p, P->z.p, mode, prev_q, prev_slot, m, P->st.p, ev, capturing);
        if (rc) return rc;
    }
    if (m == 1) {
        hipLaunchKernelGGL(spmv_p_dots_kernel, dim3(grid), dim3(VEC_BLOCK), 0, s, P->rowptr.p, P->col.p, P->val.p,
                           zsrc, prev_p[0], pv_cur, qv_cur, P->r.p, (int)n, mode, cur, P->partials.p, P->counters.p,
                           P->st.p);
    } else {
        hipLaunchKernelGGL(pupdate_kernel, dim3(grid), dim3(VEC_BLOCK), 0, s, zsrc, pv_cur, prev_p[0], prev_p[1],
                           prev_p[2], prev_p[3], m, (int)n, P->st.p);
        hipLaunchKernelGGL(spmv_dots_kernel, dim3(grid), dim3(VEC_BLOCK), 0, s, P->rowptr.p, P->col.p, P->val.p,
                           pv_cur, qv_cur, P->r.p, (int)n, mode, cur, P->partials.p, P->counters.p, P->st.p);
    }
    hipLaunchKernelGGL(update_kernel, dim3(grid), dim3(VEC_BLOCK), 0, s, P->u.p, P->r.p, pv_cur, qv_cur, (int)n, mode,
                       P->partials.p, P->counters.p, P->st.p);
    if (!capturing) HIP_TRY(hipGetLastError());
    if (ev) HIP_TRY(hipEventRecord(ev[4], s));
    return DDMGNN_OK;
}

int check_opts(const ddmgnn_solve_opts& o) {
    if (o.krylov < 0 || o.krylov > 2) return fail(DDMGNN_E_INVALID, "krylov must be FCG, PCG or CG");
    if (o.krylov == DDMGNN_FCG && (o.m_max < 1 || o.m_max > MAX_M)) return fail(DDMGNN_E_INVALID, "m_max must be in [1, 4]");
    if (!(o.rtol >= 0.0)) return fail(DDMGNN_E_INVALID, "rtol must be >= 0");
    if (o.max_it < 0) return fail(DDMGNN_E_INVALID, "max_it must be >= 0");
    if (o.precision < 0 || o.precision > 2) return fail(DDMGNN_E_INVALID, "precision must be FP64, FP32 or BF16");
    if (o.prolong < 0 || o.prolong > 1) return fail(DDMGNN_E_INVALID, "prolong must be POU or UNWEIGHTED");
    return DDMGNN_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* ddmgnn_last_error(void) { return g_err.c_str(); }
const char* ddmgnn_version(void) { return "ddmgnn 0.1 gfx950"; }
int32_t ddmgnn_max_subdomain_nodes(void) { return ddmgnn::kMaxSubNodes; }

void ddmgnn_default_opts(ddmgnn_solve_opts* o) {
    o->krylov = DDMGNN_FCG;
    o->m_max = 1;
    o->rtol = 1e-6;
    o->max_it = 10000;
    o->precision = DDMGNN_FP32;
    o->prolong = DDMGNN_PROLONG_POU;
    o->coarse = 1;
    o->check_every = 16;
    o->profile = 0;
    o->graph = 1;
}

int ddmgnn_ctx_create(void* hip_stream, ddmgnn_ctx** out) {
    if (!out) return fail(DDMGNN_E_INVALID, "null output pointer");
    auto c = std::make_unique<ddmgnn_ctx>();
    c->stream = (hipStream_t)hip_stream;
    c->launch = c->stream;
    HIP_TRY(hipGetDevice(&c->device));
    HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    HIP_TRY(c->partials.alloc(VEC_GRID));
    HIP_TRY(c->counters.alloc(4));
    HIP_TRY(hipMemset(c->counters.p, 0, 4 * sizeof(unsigned)));
    HIP_TRY(c->scalar.alloc(1));
    static_assert(sizeof(KState) <= 256, "pinned staging buffer");
    HIP_TRY(hipHostMalloc((void**)&c->host_pinned, 256, hipHostMallocDefault));
    *out = c.release();
    return DDMGNN_OK;
}

int ddmgnn_ctx_destroy(ddmgnn_ctx* ctx) {
    if (!ctx) return DDMGNN_OK;
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
    return DDMGNN_OK;
}

int ddmgnn_model_create(ddmgnn_ctx* ctx, const ddmgnn_model_desc* desc, const float* theta, int64_t n_theta,
                        ddmgnn_model** out) {
    (void)ctx;
    if (!desc || !theta || !out) return fail(DDMGNN_E_INVALID, "null argument");
    if (desc->d != D) return fail(DDMGNN_E_INVALID, "only latent width d = 10 is compiled");
    if (desc->kbar < 1) return fail(DDMGNN_E_INVALID, "kbar must be >= 1");
    const int64_t expect = (int64_t)desc->kbar * (11 * D * D + 15 * D + 1);
    if (n_theta != expect) return fail(DDMGNN_E_INVALID, "n_theta must equal kbar*(11d^2+15d+1)");
    for (int64_t i = 0; i < n_theta; ++i)
        if (!std::isfinite(theta[i])) return fail(DDMGNN_E_INVALID, "non-finite weight");
    auto m = std::make_unique<ddmgnn_model>();
    m->kbar = desc->kbar;
    m->d = desc->d;
    m->alpha = desc->alpha;
    m->theta.assign(theta, theta + n_theta);
    ddmgnn::build_mfma_blobs(m->theta.data(), m->kbar, m->mfma_steps, m->mfma_dec);
    *out = m.release();
    return DDMGNN_OK;
}

int ddmgnn_model_destroy(ddmgnn_model* m) {
    delete m;
    return DDMGNN_OK;
}

int ddmgnn_validate_problem(const ddmgnn_problem_desc* desc) {
    if (!desc) return fail(DDMGNN_E_INVALID, "null descriptor");
    std::string e = ddmgnn::validate(*desc);
    if (!e.empty()) return fail(DDMGNN_E_INVALID, e);
    return DDMGNN_OK;
}

int ddmgnn_problem_create(ddmgnn_ctx* ctx, const ddmgnn_problem_desc* desc, const ddmgnn_model* model,
                          ddmgnn_problem** out) {
    if (!ctx || !desc || !model || !out) return fail(DDMGNN_E_INVALID, "null argument");
    int rc = ddmgnn_validate_problem(desc);
    if (rc) return rc;
    auto P = std::make_unique<ddmgnn_problem>();
    P->ctx = ctx;
    std::string e = ddmgnn::build_setup(*desc, P->hs);
    if (e == "NOT_SPD") return fail(DDMGNN_E_NOT_SPD, "coarse matrix R_0 A R_0^T is not positive definite");
    if (!e.empty()) return fail(DDMGNN_E_INVALID, e);
    const auto& hs = P->hs;
    const int64_t n = hs.n, sk = hs.sk;
    const int K = hs.K;
    P->kbar = model->kbar;
    P->alpha = model->alpha;
    hipStream_t s = ctx->stream;
    HIP_TRY(P->rowptr.upload(desc->a_rowptr, n + 1, s));
    HIP_TRY(P->col.upload(desc->a_col, hs.nnz, s));
    HIP_TRY(P->val.upload(desc->a_val, hs.nnz, s));
    HIP_TRY(P->b.upload(desc->b, n, s));
    HIP_TRY(P->u0.upload(desc->u0, n, s));
    HIP_TRY(P->dirichlet.upload(desc->dirichlet, n, s));
    std::vector<int32_t> sp32(K + 1);
    for (int i = 0; i <= K; ++i) sp32[i] = (int32_t)desc->sub_ptr[i];
    HIP_TRY(P->sub_ptr.upload(sp32.data(), K + 1, s));
    HIP_TRY(P->sub_nodes.upload(desc->sub_nodes, sk, s));
    HIP_TRY(P->weights.upload(desc->weights, sk, s));
    HIP_TRY(P->work_order.upload(hs.work_order.data(), K, s));
    std::vector<int32_t> ep32(sk + 1);
    for (int64_t i = 0; i <= sk; ++i) ep32[i] = (int32_t)hs.edge_ptr[i];
    HIP_TRY(P->edge_ptr.upload(ep32.data(), sk + 1, s));
    {
        // padded by 8 entries: the chunked edge loops read up to 3 past a node's last edge
        std::vector<uint16_t> src(hs.edge_src);
        src.resize(src.size() + 8, 0);
        HIP_TRY(P->edge_src.upload(src.data(), src.size(), s));
    }
    std::vector<int32_t> np32(n + 1);
    for (int64_t i = 0; i <= n; ++i) np32[i] = (int32_t)hs.node_ptr[i];
    HIP_TRY(P->node_ptr.upload(np32.data(), n + 1, s));
    HIP_TRY(P->node_slots.upload(hs.node_slots.data(), sk, s));
    HIP_TRY(P->slot_sub.upload(hs.slot_sub.data(), sk, s));
    std::vector<double> xy64(2 * sk);
    std::vector<float> xyc32(2 * sk);
    for (int64_t k = 0; k < sk; ++k) {
        const int32_t v = desc->sub_nodes[k];
        xy64[2 * k] = desc->xy[2 * v];
        xy64[2 * k + 1] = desc->xy[2 * v + 1];
        xyc32[2 * k] = (float)hs.xyc[2 * k];
        xyc32[2 * k + 1] = (float)hs.xyc[2 * k + 1];
    }
    HIP_TRY(P->xy64.upload(xy64.data(), 2 * sk, s));
    HIP_TRY(P->xyc32.upload(xyc32.data(), 2 * sk, s));
    HIP_TRY(P->a0inv.upload(hs.a0inv.data(), (size_t)K * K, s));
    std::vector<double> th64(model->theta.begin(), model->theta.end());
    HIP_TRY(P->theta32.upload(model->theta.data(), model->theta.size(), s));
    HIP_TRY(P->theta64.upload(th64.data(), th64.size(), s));
    HIP_TRY(P->mfma_steps.upload(model->mfma_steps.data(), model->mfma_steps.size(), s));
    HIP_TRY(P->mfma_dec.upload(model->mfma_dec.data(), model->mfma_dec.size(), s));
    {
        std::vector<ddmgnn::TileNode> tiles(sk);
        for (int i = 0; i < K; ++i) {
            const int64_t b = desc->sub_ptr[i], e = desc->sub_ptr[i + 1];
            for (int64_t q = b; q < e; ++q) {
                const int32_t j = hs.tnode[q];
                const int64_t slot = b + j;
                ddmgnn::TileNode& t = tiles[q];
                t.e0 = (int32_t)hs.edge_ptr[slot];
                t.j = (uint16_t)j;
                t.deg = (uint16_t)(hs.edge_ptr[slot + 1] - hs.edge_ptr[slot]);
                t.xh = hs.xyhl[4 * slot + 0];
                t.xl = hs.xyhl[4 * slot + 1];
                t.yh = hs.xyhl[4 * slot + 2];
                t.yl = hs.xyhl[4 * slot + 3];
            }
        }
        HIP_TRY(P->tiles.upload(tiles.data(), tiles.size(), s));
        std::vector<uint32_t> er(hs.erec);
        er.resize(er.size() + 8, 0u);
        HIP_TRY(P->erec.upload(er.data(), er.size(), s));
        size_t need = 0;
        for (int i = 0; i < K; ++i) {
            const int64_t b = desc->sub_ptr[i], e = desc->sub_ptr[i + 1];
            need = std::max(need, ddmgnn::mfma_lds_need((int)(e - b), hs.edge_ptr[e] - hs.edge_ptr[b]));
        }
        P->mfma_fits = need <= ddmgnn::MFMA_LDS_LIMIT;
    }
    {
        std::vector<float> nd(hs.edge_nd);
        nd.resize(nd.size() + 8, 0.0f);
        HIP_TRY(P->edge_nd.upload(nd.data(), nd.size(), s));
    }
    HIP_TRY(P->s.alloc(K));
    HIP_TRY(P->y0.alloc(K));
    HIP_TRY(P->y.alloc(K));
    HIP_TRY(P->local.alloc(sk));
    HIP_TRY(P->u.alloc(n));
    HIP_TRY(P->r.alloc(n));
    HIP_TRY(P->z.alloc(n));
    HIP_TRY(P->ring.alloc((size_t)2 * (MAX_M + 1) * n));
    std::vector<double*> rp(2 * (MAX_M + 1));
    for (int i = 0; i < 2 * (MAX_M + 1); ++i) rp[i] = P->ring.p + (size_t)i * n;
    HIP_TRY(P->ring_ptrs.upload(rp.data(), rp.size(), s));
    HIP_TRY(P->st.alloc(1));
    HIP_TRY(P->partials.alloc((size_t)(MAX_M + 1) * VEC_GRID));
    HIP_TRY(P->counters.alloc(4));
    HIP_TRY(hipMemsetAsync(P->counters.p, 0, 4 * sizeof(unsigned), s));
    HIP_TRY(hipMemsetAsync(P->st.p, 0, sizeof(KState), s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = P.release();
    return DDMGNN_OK;
}

int ddmgnn_problem_destroy(ddmgnn_problem* P) {
    delete P;
    return DDMGNN_OK;
}

int ddmgnn_problem_sizes(const ddmgnn_problem* P, int64_t* n, int64_t* nnz, int32_t* k, int64_t* sum_k,
                         int64_t* n_edges) {
    if (!P) return fail(DDMGNN_E_INVALID, "null problem");
    if (n) *n = P->hs.n;
    if (nnz) *nnz = P->hs.nnz;
    if (k) *k = P->hs.K;
    if (sum_k) *sum_k = P->hs.sk;
    if (n_edges) *n_edges = P->hs.n_edges;
    return DDMGNN_OK;
}

int ddmgnn_setup_local_graph(const ddmgnn_problem_desc* desc, int32_t sub, int32_t* rowptr, int32_t* col,
                             int64_t* n_edges_sub) {
    int rc = ddmgnn_validate_problem(desc);
    if (rc) return rc;
    if (sub < 0 || sub >= desc->n_sub) return fail(DDMGNN_E_INVALID, "sub-mesh index out of range");
    ddmgnn::HostSetup hs;
    ddmgnn::build_local_graphs(*desc, hs);
    const int64_t b = desc->sub_ptr[sub], e = desc->sub_ptr[sub + 1];
    const int64_t e0 = hs.edge_ptr[b], e1 = hs.edge_ptr[e];
    if (n_edges_sub) *n_edges_sub = e1 - e0;
    if (rowptr)
        for (int64_t k = b; k <= e; ++k) rowptr[k - b] = (int32_t)(hs.edge_ptr[k] - e0);
    if (col)
        for (int64_t q = e0; q < e1; ++q) col[q - e0] = hs.edge_src[q];
    return DDMGNN_OK;
}

int ddmgnn_setup_coarse(const ddmgnn_problem_desc* desc, double* a0, double* a0inv) {
    int rc = ddmgnn_validate_problem(desc);
    if (rc) return rc;
    ddmgnn::HostSetup hs;
    std::string e = ddmgnn::build_setup(*desc, hs);
    if (!hs.a0.empty() && a0) std::memcpy(a0, hs.a0.data(), hs.a0.size() * sizeof(double));
    if (e == "NOT_SPD") return fail(DDMGNN_E_NOT_SPD, "coarse matrix R_0 A R_0^T is not positive definite");
    if (!e.empty()) return fail(DDMGNN_E_INVALID, e);
    if (a0inv) std::memcpy(a0inv, hs.a0inv.data(), hs.a0inv.size() * sizeof(double));
    return DDMGNN_OK;
}

int ddmgnn_spmv(ddmgnn_ctx* ctx, ddmgnn_problem* P, const double* x, double* y) {
    if (!ctx || !P || !x || !y) return fail(DDMGNN_E_INVALID, "null argument");
    hipLaunchKernelGGL(spmv_kernel, dim3(vec_grid(P->hs.n)), dim3(VEC_BLOCK), 0, ctx->stream, P->rowptr.p, P->col.p,
                       P->val.p, x, y, (int)P->hs.n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DDMGNN_OK;
}

int ddmgnn_dot(ddmgnn_ctx* ctx, int64_t n, const double* x, const double* y, double* out) {
    if (!ctx || !out || n < 0 || (n > 0 && (!x || !y))) return fail(DDMGNN_E_INVALID, "invalid argument");
    if (n == 0) {
        *out = 0.0;
        return DDMGNN_OK;
    }
    hipLaunchKernelGGL(dot_kernel, dim3(vec_grid(n)), dim3(VEC_BLOCK), 0, ctx->stream, x, y, n, ctx->partials.p,
                       ctx->counters.p, ctx->scalar.p);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ctx->host_pinned, ctx->scalar.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *out = ctx->host_pinned[0];
    return DDMGNN_OK;
}

int ddmgnn_dss_forward(ddmgnn_ctx* ctx, ddmgnn_problem* P, int32_t precision, const double* c, double* out) {
    if (!ctx || !P || !c || !out) return fail(DDMGNN_E_INVALID, "null argument");
    if (precision < 0 || precision > 2) return fail(DDMGNN_E_INVALID, "bad precision");
    int rc = launch_dss(P, precision, false, nullptr, c, out, nullptr);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DDMGNN_OK;
}

int ddmgnn_precond_apply(ddmgnn_ctx* ctx, ddmgnn_problem* P, const ddmgnn_solve_opts* opts, const double* r,
                         double* z) {
    if (!ctx || !P || !opts || !r || !z) return fail(DDMGNN_E_INVALID, "null argument");
    if (r == z) return fail(DDMGNN_E_INVALID, "r and z must not alias");
    int rc = check_opts(*opts);
    if (rc) return rc;
    rc = enqueue_apply(P, *opts, r, z, -1, nullptr, nullptr, 0, nullptr);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DDMGNN_OK;
}

int ddmgnn_apply_intermediates(ddmgnn_ctx* ctx, ddmgnn_problem* P, double* s, double* y0, double* y,
                               double* local) {
    if (!ctx || !P) return fail(DDMGNN_E_INVALID, "null argument");
    hipStream_t st = ctx->stream;
    const int K = P->hs.K;
    if (s) HIP_TRY(hipMemcpyAsync(s, P->s.p, K * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (y0) HIP_TRY(hipMemcpyAsync(y0, P->y0.p, K * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (y) HIP_TRY(hipMemcpyAsync(y, P->y.p, K * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (local) HIP_TRY(hipMemcpyAsync(local, P->local.p, P->hs.sk * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return DDMGNN_OK;
}

int ddmgnn_solve(ddmgnn_ctx* ctx, ddmgnn_problem* P, const ddmgnn_solve_opts* opts, double* u_out,
                 ddmgnn_stats* stats) {
    if (!ctx || !P || !opts || !u_out) return fail(DDMGNN_E_INVALID, "null argument");
    int rc = check_opts(*opts);
    if (rc) return rc;
    const ddmgnn_solve_opts& o = *opts;
    hipStream_t s = ctx->stream;
    const int64_t n = P->hs.n;
    const int grid = vec_grid(n);
    const int nring = (o.krylov == DDMGNN_FCG ? o.m_max : 1) + 1;
    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    HIP_TRY(hipMemcpyAsync(P->u.p, P->u0.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipEventRecord(ev0, s));
    hipLaunchKernelGGL(init_kernel, dim3(grid), dim3(VEC_BLOCK), 0, s, P->rowptr.p, P->col.p, P->val.p, P->b.p,
                       P->u.p, P->r.p, P->ring_ptrs.p, 2 * (MAX_M + 1), (int)n, o.rtol, o.max_it, P->partials.p,
                       P->counters.p, P->st.p);
    HIP_TRY(hipGetLastError());
    KState host_state{};
    // Iterations between host polls of the converged flag. With graph replay
    // the chunk length is a multiple of the direction-ring length, so every
    // chunk has the same kernels and pointers and one captured graph serves all.
    int check = std::max(1, o.check_every);
    const bool use_graph = o.graph && !o.profile;
    if (use_graph) check = ((check + nring - 1) / nring) * nring;
    // Profiling: 5 events per iteration of a chunk (before DSS, after DSS,
    // after coarse, after prolong, after the Krylov kernels).
    std::vector<hipEvent_t> pev;
    if (o.profile) {
        pev.resize((size_t)check * 5);
        for (auto& e : pev) HIP_TRY(hipEventCreate(&e));
    }
    hipGraphExec_t gexec = nullptr;
    if (use_graph) {
        const uint64_t key = ((uint64_t)o.krylov << 40) | ((uint64_t)o.m_max << 32) | ((uint64_t)o.precision << 24) |
                             ((uint64_t)o.prolong << 16) | ((uint64_t)o.coarse << 8) | (uint64_t)check;
        if (!P->graph_exec || P->graph_key != key) {
            if (P->graph_exec) {
                (void)hipGraphExecDestroy(P->graph_exec);
                P->graph_exec = nullptr;
            }
            hipGraph_t g = nullptr;
            if (o.krylov != DDMGNN_CG)
                if (int prc = prepare_dss(P, o.precision)) return prc;
            // Capture on the context's own stream (the caller's stream may be the
            // null stream, which cannot be captured); the graph runs on s.
            hipStream_t cs_stream = ctx->cap;
            HIP_TRY(hipStreamBeginCapture(cs_stream, hipStreamCaptureModeRelaxed));
            ctx->launch = cs_stream;
            int crc = 0;
            for (int c = 0; c < check && crc == 0; ++c) crc = enqueue_iteration(P, o, c, nullptr, true);
            ctx->launch = ctx->stream;
            hipError_t ce = hipStreamEndCapture(cs_stream, &g);
            if (crc || ce != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
                if (hipStreamIsCapturing(cs_stream, &cst) == hipSuccess && cst != hipStreamCaptureStatusNone) {
                    hipGraph_t g2 = nullptr;
                    (void)hipStreamEndCapture(cs_stream, &g2);
                    if (g2) (void)hipGraphDestroy(g2);
                }
                if (crc) return crc;
                HIP_TRY(ce);
            }
            HIP_TRY(hipGetLastError());
            hipError_t ie = hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(ie);
            P->graph_key = key;
        }
        gexec = P->graph_exec;
    }
    double t_dss = 0, t_coarse = 0, t_prolong = 0, t_krylov = 0;
    int n_dss = 0;
    int it = 0;
    bool done = false;
    while (!done) {
        const int it_chunk0 = it;
        int n_chunk = 0;
        if (gexec) {
            HIP_TRY(hipGraphLaunch(gexec, s));
            it += check;
            n_chunk = check;
        } else {
            for (int c = 0; c < check && it < o.max_it; ++c, ++it, ++n_chunk) {
                rc = enqueue_iteration(P, o, it, o.profile ? &pev[(size_t)c * 5] : nullptr);
                if (rc) return rc;
            }
        }
        HIP_TRY(hipMemcpyAsync(ctx->host_pinned, P->st.p, sizeof(KState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(&host_state, ctx->host_pinned, sizeof(KState));
        done = host_state.done || it >= o.max_it;
        if (o.profile) {
            // iterations it_chunk0 .. host_state.it-1 did work; later ones exited early
            const int worked = std::min(n_chunk, std::max(0, host_state.it - it_chunk0));
            for (int c = 0; c < worked; ++c) {
                hipEvent_t* ev = &pev[(size_t)c * 5];
                float a = 0, b = 0, cc = 0, d = 0;
                HIP_TRY(hipEventElapsedTime(&a, ev[0], ev[1]));
                HIP_TRY(hipEventElapsedTime(&b, ev[1], ev[2]));
                HIP_TRY(hipEventElapsedTime(&cc, ev[2], ev[3]));
                HIP_TRY(hipEventElapsedTime(&d, ev[3], ev[4]));
                t_dss += a;
                t_coarse += b;
                t_prolong += cc;
                t_krylov += d;
                if (o.krylov != DDMGNN_CG) ++n_dss;
            }
        }
    }
    for (auto& e : pev) (void)hipEventDestroy(e);
    HIP_TRY(hipEventRecord(ev1, s));
    // true residual |b - A u| / |r_0|
    hipLaunchKernelGGL(resid_kernel, dim3(grid), dim3(VEC_BLOCK), 0, s, P->rowptr.p, P->col.p, P->val.p, P->b.p,
                       P->u.p, (int)n, ctx->partials.p, ctx->counters.p, ctx->scalar.p);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(u_out, P->u.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->host_pinned, ctx->scalar.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double tr = ctx->host_pinned[0];
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    HIP_TRY(hipEventDestroy(ev0));
    HIP_TRY(hipEventDestroy(ev1));
    const bool converged = host_state.status == 0 && host_state.rel <= o.rtol;
    if (stats) {
        stats->iterations = host_state.it;
        stats->converged = converged;
        stats->rel_residual = host_state.rel;
        stats->true_rel_residual = host_state.r0n > 0 ? std::sqrt(tr) / host_state.r0n : 0.0;
        stats->solve_ms = ms;
        stats->dss_launches = n_dss;
        stats->dss_ms = t_dss;
        stats->coarse_ms = t_coarse;
        stats->prolong_ms = t_prolong;
        stats->krylov_ms = t_krylov;
        stats->dss_kernel = o.precision == DDMGNN_FP64 ? 0 : (o.precision == DDMGNN_BF16 && P->mfma_fits ? 2 : 1);
    }
    if (host_state.status) return fail(host_state.status, "Krylov breakdown or non-finite residual");
    if (!converged) return fail(DDMGNN_E_MAXIT, "not converged within max_it");
    return DDMGNN_OK;
}

int ddmgnn_expand_overlap(int64_t n_nodes, int64_t n_tri, const int32_t* tri, const int32_t* part, int32_t n_part,
                          int32_t delta, int64_t** sub_ptr_out, int32_t** sub_nodes_out) {
    if (n_nodes <= 0 || n_tri <= 0 || !tri || !part || n_part <= 0 || delta < 0 || !sub_ptr_out || !sub_nodes_out)
        return fail(DDMGNN_E_INVALID, "invalid argument");
    for (int64_t t = 0; t < 3 * n_tri; ++t)
        if (tri[t] < 0 || tri[t] >= n_nodes) return fail(DDMGNN_E_INVALID, "triangle node id out of range");
    for (int64_t i = 0; i < n_nodes; ++i)
        if (part[i] < 0 || part[i] >= n_part) return fail(DDMGNN_E_INVALID, "part id out of range");
    std::vector<int64_t> sp;
    std::vector<int32_t> sn;
    ddmgnn::expand_overlap(n_nodes, n_tri, tri, part, n_part, delta, sp, sn);
    auto* a = (int64_t*)std::malloc(sp.size() * sizeof(int64_t));
    auto* b = (int32_t*)std::malloc(std::max<size_t>(1, sn.size()) * sizeof(int32_t));
    if (!a || !b) {
        std::free(a);
        std::free(b);
        return fail(DDMGNN_E_NOMEM, "host allocation failed");
    }
    std::memcpy(a, sp.data(), sp.size() * sizeof(int64_t));
    std::memcpy(b, sn.data(), sn.size() * sizeof(int32_t));
    *sub_ptr_out = a;
    *sub_nodes_out = b;
    return DDMGNN_OK;
}

int ddmgnn_pou_weights(int64_t n_nodes, const uint8_t* dirichlet, int32_t n_sub, const int64_t* sub_ptr,
                       const int32_t* sub_nodes, double* weights_out) {
    if (n_nodes <= 0 || !dirichlet || n_sub <= 0 || !sub_ptr || !sub_nodes || !weights_out)
        return fail(DDMGNN_E_INVALID, "invalid argument");
    std::vector<int32_t> mult(n_nodes, 0);
    for (int64_t k = 0; k < sub_ptr[n_sub]; ++k) {
        if (sub_nodes[k] < 0 || sub_nodes[k] >= n_nodes) return fail(DDMGNN_E_INVALID, "node id out of range");
        mult[sub_nodes[k]]++;
    }
    for (int64_t k = 0; k < sub_ptr[n_sub]; ++k) {
        const int32_t v = sub_nodes[k];
        weights_out[k] = dirichlet[v] ? 0.0 : 1.0 / (double)mult[v];
    }
    return DDMGNN_OK;
}

void ddmgnn_free(void* p) { std::free(p); }

}  // extern "C"
