// Device factorisation: the exact local solvers of DDM-LU (eq. (7); the
// paper's comparator of Tables I and III) and the coarse level (Sec. III.A
// step 1). For every sub-mesh i the dense local matrix A_i = R_i A R_i^T is
// assembled from the CSR matrix, and the coarse matrix A_0 = R_0 A R_0^T
// from the CSR matrix and the partition-of-unity weights; both are inverted
// in place, so that every apply is one GEMV per sub-mesh (lu_local_kernel) and
// one for the coarse level (coarse_kernel).
//
// Inversion: blocked Gauss-Jordan without pivoting, which is safe for a
// symmetric positive definite matrix (every pivot block is a diagonal block
// of a Schur complement, itself SPD). For pivot block P (GJ_W rows and
// columns) and the remaining indices R, one step replaces
//   A_PP <- A_PP^{-1},             A_PR <- A_PP^{-1} A_PR,
//   A_RP <- -A_RP A_PP^{-1},       A_RR <- A_RR - A_RP A_PP^{-1} A_PR,
// and after the last block the matrix holds its inverse (the in-place
// inversion of Gauss-Jordan elimination, one block of pivots at a time).
//
// A batch of matrices (the K local matrices, or the single coarse matrix)
// takes four launches per pivot step over the whole device: the pivot block
// inverses (one workgroup per matrix), the new pivot rows (workgroups over
// column chunks of every matrix), the update of every 64 x 64 tile of every
// matrix, and the new pivot columns with the pivot block. A workgroup finds
// its matrix by binary search in a prefix of per-matrix workgroup counts;
// matrices already finished at that step return at once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"

namespace ddmgnn {

namespace {

constexpr int GJ_THREADS = 256;
constexpr int GJ_W = 64;  // pivot block width
constexpr int GJ_T = 64;  // rows and columns of a tile of the trailing update (4 x 4 per thread)
static_assert(GJ_T == 16 * 4 && GJ_THREADS == 16 * 16, "tile of 4 x 4 outputs per thread");

// Binary search of node g in the ascending slice s[0..k); -1 when absent.
__device__ inline int find_local(const int32_t* __restrict__ s, int k, int32_t g) {
    int lo = 0, hi = k;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s[mid] < g) lo = mid + 1;
        else hi = mid;
    }
    return lo < k && s[lo] == g ? lo : -1;
}

// A_i = R_i A R_i^T of sub-mesh blockIdx.x, dense, sub-mesh i at off[i] with
// row stride (off[i + 1] - off[i]) / k_i (the pad column stays zero).
__global__ __launch_bounds__(GJ_THREADS) void lu_assemble_kernel(const int32_t* __restrict__ rowptr,
                                                                  const int32_t* __restrict__ col,
                                                                  const double* __restrict__ val,
                                                                  const int64_t* __restrict__ sub_ptr,
                                                                  const int32_t* __restrict__ sub_nodes,
                                                                  const int64_t* __restrict__ off,
                                                                  double* __restrict__ inv) {
    const int i = blockIdx.x;
    const int64_t b = sub_ptr[i];
    const int k = (int)(sub_ptr[i + 1] - b);
    if (k == 0) return;
    const int64_t ld = (off[i + 1] - off[i]) / k;  // row stride of the stored inverse
    double* M = inv + off[i];
    const int32_t* s = sub_nodes + b;
    for (int64_t e = threadIdx.x; e < (int64_t)k * ld; e += GJ_THREADS) M[e] = 0.0;
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += GJ_THREADS) {
        const int32_t g = s[j];
        for (int32_t e = rowptr[g]; e < rowptr[g + 1]; ++e) {
            const int q = find_local(s, k, col[e]);
            if (q >= 0) M[(int64_t)j * ld + q] = val[e];
        }
    }
}

// A_0 = Z^T A Z (column i of Z is R_i^T D_i R_i 1): row i sums w_a A[g_a][m] w_b
// over the slots a of sub-mesh i, the nonzeros (g_a, m) of A and the slots b
// of node m (sub-mesh j = slot_sub[b]). One workgroup builds one row. A row has
// few nonzero columns (the sub-meshes that touch sub-mesh i or its neighbours),
// so the workgroup first marks them in an LDS bitmap, then every thread sums a
// contiguous chunk of the slots into its own accumulator per marked column, and
// the chunks' sums are added in thread order: the bits do not depend on
// scheduling. A row with more than CA_MAXJ columns, or K above CA_MAXK, is
// summed by one thread in slot, nonzero and membership order.
constexpr int CA_THREADS = 256;
constexpr int CA_MAXK = 16384;  // columns covered by the LDS bitmap
constexpr int CA_MAXJ = 32;     // nonzero columns per row held in LDS
__global__ __launch_bounds__(CA_THREADS) void coarse_assemble_kernel(const int32_t* __restrict__ rowptr,
                                                                     const int32_t* __restrict__ col,
                                                                     const double* __restrict__ val,
                                                                     const int32_t* __restrict__ sub_ptr,
                                                                     const int32_t* __restrict__ sub_nodes,
                                                                     const double* __restrict__ weights,
                                                                     const int32_t* __restrict__ node_ptr,
                                                                     const int32_t* __restrict__ node_slots,
                                                                     const int32_t* __restrict__ slot_sub, int K,
                                                                     double* __restrict__ a0) {
    __shared__ uint32_t bits[CA_MAXK / 32];
    __shared__ int32_t wpre[CA_MAXK / 32 + 1];
    __shared__ int32_t cols[CA_MAXJ];
    __shared__ double acc[CA_MAXJ][CA_THREADS + 1];
    const int i = blockIdx.x, t = threadIdx.x;
    double* row = a0 + (size_t)i * K;
    for (int j = t; j < K; j += CA_THREADS) row[j] = 0.0;
    const int s0 = sub_ptr[i], s1 = sub_ptr[i + 1];
    if (K <= CA_MAXK) {  // uniform over the workgroup
        const int W = (K + 31) / 32;
        for (int w = t; w < W; w += CA_THREADS) bits[w] = 0u;
        __syncthreads();
        for (int a = s0 + t; a < s1; a += CA_THREADS) {
            if (weights[a] == 0.0) continue;
            const int32_t g = sub_nodes[a];
            for (int32_t e = rowptr[g]; e < rowptr[g + 1]; ++e) {
                const int32_t m = col[e];
                for (int32_t q = node_ptr[m]; q < node_ptr[m + 1]; ++q) {
                    const int32_t j = slot_sub[node_slots[q]];
                    atomicOr(&bits[j >> 5], 1u << (j & 31));
                }
            }
        }
        __syncthreads();
        if (t == 0) {
            int c = 0;
            for (int w = 0; w < W; ++w) {
                wpre[w] = c;
                c += __popc(bits[w]);
            }
            wpre[W] = c;
        }
        __syncthreads();
        const int nj = wpre[W];
        if (nj <= CA_MAXJ) {  // uniform
            for (int w = t; w < W; w += CA_THREADS) {
                uint32_t b = bits[w];
                for (int c = wpre[w]; b; ++c, b &= b - 1u) cols[c] = w * 32 + __ffs((int)b) - 1;
            }
            for (int c = 0; c < nj; ++c) acc[c][t] = 0.0;
            const int per = (s1 - s0 + CA_THREADS - 1) / CA_THREADS;
            const int a_lo = s0 + t * per, a_hi = min(s1, a_lo + per);
            for (int a = a_lo; a < a_hi; ++a) {
                const double wa = weights[a];
                if (wa == 0.0) continue;
                const int32_t g = sub_nodes[a];
                for (int32_t e = rowptr[g]; e < rowptr[g + 1]; ++e) {
                    const int32_t m = col[e];
                    const double v = val[e] * wa;
                    for (int32_t q = node_ptr[m]; q < node_ptr[m + 1]; ++q) {
                        const int32_t b = node_slots[q], j = slot_sub[b];
                        const int c = wpre[j >> 5] + __popc(bits[j >> 5] & ((1u << (j & 31)) - 1u));
                        acc[c][t] += v * weights[b];
                    }
                }
            }
            __syncthreads();
            for (int c = t; c < nj; c += CA_THREADS) {
                double sum = 0.0;
                for (int u = 0; u < CA_THREADS; ++u) sum += acc[c][u];
                row[cols[c]] = sum;
            }
            return;
        }
    }
    __syncthreads();  // the row is zero before the single-thread sum writes it
    if (t != 0) return;
    for (int a = s0; a < s1; ++a) {
        const double wa = weights[a];
        if (wa == 0.0) continue;
        const int32_t g = sub_nodes[a];
        for (int32_t e = rowptr[g]; e < rowptr[g + 1]; ++e) {
            const int32_t m = col[e];
            const double v = val[e] * wa;
            for (int32_t q = node_ptr[m]; q < node_ptr[m + 1]; ++q) {
                const int32_t b = node_slots[q];
                row[slot_sub[b]] += v * weights[b];
            }
        }
    }
}

// Exact symmetry of A_0: both triangles take the mean of the two sums; the
// diagonal is kept in diag0 (the reference of the pivot test).
__global__ __launch_bounds__(256) void coarse_symmetrise_kernel(double* __restrict__ a0, int K,
                                                                double* __restrict__ diag0) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)K * K) return;
    const int i = (int)(e / K), j = (int)(e % K);
    if (j == i) diag0[i] = a0[e];
    if (j <= i) return;
    const double m = 0.5 * (a0[(size_t)i * K + j] + a0[(size_t)j * K + i]);
    a0[(size_t)i * K + j] = m;
    a0[(size_t)j * K + i] = m;
}

// One matrix of a batch: order k, row stride ld, entries at M.
struct GjMat {
    double* M;
    int k;
    int64_t ld;
};
struct GjBatch {
    double* base;
    const int64_t* off;     // [nm + 1] matrix m at base + off[m], row stride (off[m + 1] - off[m]) / k_m
    const int32_t* order;   // [nm] k_m
    int nm;
    const int32_t* cprefix; // [nm + 1] prefix of ceil(k_m / GJ_THREADS) (row and column workgroups)
    const int32_t* tprefix; // [nm + 1] prefix of ceil(k_m / GJ_T)^2 (tile workgroups)
    double* dinv;           // [nm][GJ_W][GJ_W] pivot block inverses
    double* pr;             // matrix m's new pivot rows at pr + GJ_W * prow[m], row stride k_m
    const int64_t* prow;    // [nm + 1] prefix of k_m
    const double* diag0;    // optional: original diagonal (pivot test reference) of matrix 0
    int* status;            // bit 0: a pivot not positive (or below GJ_REL of diag0)
};
__device__ inline GjMat gj_mat(const GjBatch& b, int m) {
    const int k = b.order[m];
    return {b.base + b.off[m], k, k > 0 ? (b.off[m + 1] - b.off[m]) / k : 0};
}
// Matrix of workgroup w in a prefix of per-matrix workgroup counts (the last m
// with prefix[m] <= w), and w's index within that matrix.
__device__ inline int gj_find(const int32_t* prefix, int nm, int w, int* local) {
    int lo = 0, hi = nm;
    while (lo + 1 < hi) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= w) lo = mid;
        else hi = mid;
    }
    *local = w - prefix[lo];
    return lo;
}

// A pivot is accepted when it is positive and, for the coarse matrix, above
// GJ_REL times its original diagonal entry: a singular or nearly singular A_0
// is refused instead of inverted.
constexpr double GJ_REL = 1e-12;

__global__ __launch_bounds__(GJ_THREADS) void gj_pivot_kernel(GjBatch b, int pb) {
    __shared__ double D[GJ_W][GJ_W + 1];
    const int m = blockIdx.x;
    const GjMat A = gj_mat(b, m);
    if (pb >= A.k) return;
    const int t = threadIdx.x, w = min(GJ_W, A.k - pb);
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) {
        const int r = e / GJ_W, c = e % GJ_W;
        D[r][c] = r < w && c < w ? A.M[(int64_t)(pb + r) * A.ld + pb + c] : 0.0;
    }
    __syncthreads();
    constexpr int PER = GJ_W * GJ_W / GJ_THREADS;
    for (int q = 0; q < w; ++q) {
        const double dq = D[q][q];
        const double floor = b.diag0 ? GJ_REL * fabs(b.diag0[pb + q]) : 0.0;
        if (t == 0 && (!(dq > floor) || !isfinite(dq))) atomicOr(b.status, 1);
        const double piv = 1.0 / dq;
        double nv[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = t + u * GJ_THREADS, r = e / GJ_W, c = e % GJ_W;
            double v = D[r][c];
            if (r == q && c == q) v = piv;
            else if (r == q) v = v * piv;
            else if (c == q) v = -v * piv;
            else v = fma(-D[r][q] * piv, D[q][c], v);
            nv[u] = v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = t + u * GJ_THREADS;
            if (e / GJ_W < w && e % GJ_W < w) D[e / GJ_W][e % GJ_W] = nv[u];
        }
        __syncthreads();
    }
    double* di = b.dinv + (size_t)m * GJ_W * GJ_W;
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) di[e] = D[e / GJ_W][e % GJ_W];
}

// A_PR(new) = dinv A_PR, one column per thread, into pr (GJ_W x k): the pivot
// rows of the matrix are replaced only after the tile update, which reads the
// old A_RP from the matrix and the new A_PR from pr.
__global__ __launch_bounds__(GJ_THREADS) void gj_rows_kernel(GjBatch b, int pb) {
    __shared__ double D[GJ_W][GJ_W + 1];
    int cb = 0;
    const int m = gj_find(b.cprefix, b.nm, blockIdx.x, &cb);
    const GjMat A = gj_mat(b, m);
    if (pb >= A.k) return;
    const int t = threadIdx.x, w = min(GJ_W, A.k - pb);
    const double* di = b.dinv + (size_t)m * GJ_W * GJ_W;
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) D[e / GJ_W][e % GJ_W] = di[e];
    __syncthreads();
    const int j = cb * GJ_THREADS + t;
    if (j >= A.k) return;
    double* pr = b.pr + (size_t)GJ_W * b.prow[m];
    double x[GJ_W];
#pragma unroll
    for (int r = 0; r < GJ_W; ++r) x[r] = r < w ? A.M[(int64_t)(pb + r) * A.ld + j] : 0.0;
    for (int r = 0; r < w; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < GJ_W; ++c) acc = fma(D[r][c], x[c], acc);
        pr[(size_t)r * A.k + j] = acc;
    }
}

// A_RR -= A_RP(old) A_PR(new) on one GJ_T x GJ_T tile per workgroup.
__global__ __launch_bounds__(GJ_THREADS) void gj_tiles_kernel(GjBatch b, int pb) {
    __shared__ double F[GJ_T][GJ_W + 1];
    __shared__ double R[GJ_W][GJ_T + 1];
    int tl = 0;
    const int m = gj_find(b.tprefix, b.nm, blockIdx.x, &tl);
    const GjMat A = gj_mat(b, m);
    if (pb >= A.k) return;
    const int t = threadIdx.x, w = min(GJ_W, A.k - pb), pe = pb + w;
    const int nt = (A.k + GJ_T - 1) / GJ_T;
    const int i0 = (tl / nt) * GJ_T, j0 = (tl % nt) * GJ_T;
    const double* pr = b.pr + (size_t)GJ_W * b.prow[m];
    for (int e = t; e < GJ_T * GJ_W; e += GJ_THREADS) {
        const int r = e / GJ_W, c = e % GJ_W, i = i0 + r;
        F[r][c] = i < A.k && (i < pb || i >= pe) && c < w ? A.M[(int64_t)i * A.ld + pb + c] : 0.0;
    }
    for (int e = t; e < GJ_W * GJ_T; e += GJ_THREADS) {
        const int r = e / GJ_T, c = e % GJ_T, j = j0 + c;
        R[r][c] = r < w && j < A.k && (j < pb || j >= pe) ? pr[(size_t)r * A.k + j] : 0.0;
    }
    __syncthreads();
    const int ty = t / 16, tx = t % 16;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    for (int p = 0; p < w; ++p) {
        double f[4], g[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) f[a] = F[ty * 4 + a][p];
#pragma unroll
        for (int c = 0; c < 4; ++c) g[c] = R[p][tx * 4 + c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] = fma(f[a], g[c], acc[a][c]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + ty * 4 + a;
        if (i >= A.k || (i >= pb && i < pe)) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tx * 4 + c;
            if (j >= A.k || (j >= pb && j < pe)) continue;
            A.M[(int64_t)i * A.ld + j] -= acc[a][c];
        }
    }
}

// A_RP <- -A_RP(old) dinv (one row per thread), the pivot rows <- pr and the
// pivot block <- dinv.
__global__ __launch_bounds__(GJ_THREADS) void gj_cols_kernel(GjBatch b, int pb) {
    __shared__ double D[GJ_W][GJ_W + 1];
    int cb = 0;
    const int m = gj_find(b.cprefix, b.nm, blockIdx.x, &cb);
    const GjMat A = gj_mat(b, m);
    if (pb >= A.k) return;
    const int t = threadIdx.x, w = min(GJ_W, A.k - pb), pe = pb + w;
    const double* di = b.dinv + (size_t)m * GJ_W * GJ_W;
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) D[e / GJ_W][e % GJ_W] = di[e];
    __syncthreads();
    const int i = cb * GJ_THREADS + t;
    if (i >= A.k) return;
    const double* pr = b.pr + (size_t)GJ_W * b.prow[m];
    double* row = A.M + (int64_t)i * A.ld;
    if (i >= pb && i < pe) {
        const int r = i - pb;
        for (int j = 0; j < A.k; ++j) row[j] = j >= pb && j < pe ? D[r][j - pb] : pr[(size_t)r * A.k + j];
        return;
    }
    double f[GJ_W];
#pragma unroll
    for (int c = 0; c < GJ_W; ++c) f[c] = c < w ? row[pb + c] : 0.0;
    for (int c = 0; c < w; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < GJ_W; ++q) acc = fma(f[q], D[q][c], acc);
        row[pb + c] = -acc;
    }
}

}  // namespace

GjPlan::GjPlan(const std::vector<int32_t>& k) {
    const int nm = (int)k.size();
    order = k;
    cprefix.assign((size_t)nm + 1, 0);
    tprefix.assign((size_t)nm + 1, 0);
    prow.assign((size_t)nm + 1, 0);
    for (int m = 0; m < nm; ++m) {
        const int64_t nt = (k[m] + GJ_T - 1) / GJ_T;
        cprefix[m + 1] = cprefix[m] + (k[m] + GJ_THREADS - 1) / GJ_THREADS;
        tiles += nt * nt;
        tprefix[m + 1] = (int32_t)std::min<int64_t>(tiles, INT32_MAX);
        prow[m + 1] = prow[m] + k[m];
        max_k = std::max(max_k, k[m]);
    }
}

size_t GjPlan::scratch_doubles() const { return order.size() * GJ_W * GJ_W + (size_t)GJ_W * prow.back(); }

hipError_t launch_gj_invert(const GjPlan& plan, const GjPlanDev& dev, double* base, const int64_t* off,
                            double* scratch, const double* diag0, int* status, hipStream_t s) {
    const int nm = (int)plan.order.size();
    if (nm == 0) return hipSuccess;
    GjBatch b{base, off, dev.order, nm, dev.cprefix, dev.tprefix, scratch, scratch + (size_t)nm * GJ_W * GJ_W,
              dev.prow, diag0, status};
    const unsigned nc = (unsigned)plan.cprefix.back(), ntl = (unsigned)plan.tprefix.back();
    if (plan.tiles * GJ_THREADS >= (int64_t)1 << 32) return hipErrorInvalidConfiguration;  // grid limit
    for (int pb = 0; pb < plan.max_k; pb += GJ_W) {
        hipLaunchKernelGGL(gj_pivot_kernel, dim3(nm), dim3(GJ_THREADS), 0, s, b, pb);
        hipLaunchKernelGGL(gj_rows_kernel, dim3(nc), dim3(GJ_THREADS), 0, s, b, pb);
        hipLaunchKernelGGL(gj_tiles_kernel, dim3(ntl), dim3(GJ_THREADS), 0, s, b, pb);
        hipLaunchKernelGGL(gj_cols_kernel, dim3(nc), dim3(GJ_THREADS), 0, s, b, pb);
    }
    return hipGetLastError();
}

hipError_t launch_lu_assemble(const int32_t* rowptr, const int32_t* col, const double* val, const int64_t* sub_ptr,
                              const int32_t* sub_nodes, const int64_t* off, double* inv, int n_sub, hipStream_t s) {
    if (n_sub <= 0) return hipSuccess;
    hipLaunchKernelGGL(lu_assemble_kernel, dim3(n_sub), dim3(GJ_THREADS), 0, s, rowptr, col, val, sub_ptr,
                       sub_nodes, off, inv);
    return hipGetLastError();
}

hipError_t launch_coarse_assemble(const int32_t* rowptr, const int32_t* col, const double* val,
                                  const int32_t* sub_ptr, const int32_t* sub_nodes, const double* weights,
                                  const int32_t* node_ptr, const int32_t* node_slots, const int32_t* slot_sub, int K,
                                  double* a0, double* diag0, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(coarse_assemble_kernel, dim3(K), dim3(CA_THREADS), 0, s, rowptr, col, val, sub_ptr,
                       sub_nodes, weights, node_ptr, node_slots, slot_sub, K, a0);
    const int64_t kk = (int64_t)K * K;
    hipLaunchKernelGGL(coarse_symmetrise_kernel, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, s, a0, K, diag0);
    return hipGetLastError();
}

}  // namespace ddmgnn
