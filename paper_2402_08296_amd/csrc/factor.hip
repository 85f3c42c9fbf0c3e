// Device factorisation of the exact local solvers of DDM-LU (eq. (7); the
// paper's comparator of Tables I and III): for every sub-mesh i the dense
// local matrix A_i = R_i A R_i^T is assembled from the CSR matrix and inverted
// in place, so that every apply is one GEMV per sub-mesh (lu_local_kernel).
//
// Inversion: blocked Gauss-Jordan without pivoting, which is safe for a
// symmetric positive definite matrix (every pivot block is a diagonal block
// of a Schur complement of A_i, itself SPD). For pivot block P (GJ_W rows and
// columns) and the remaining indices R, one step replaces
//   A_PP <- A_PP^{-1},             A_PR <- A_PP^{-1} A_PR,
//   A_RP <- -A_RP A_PP^{-1},       A_RR <- A_RR - A_RP A_PP^{-1} A_PR,
// and after the last block the matrix holds A_i^{-1} (the in-place inversion
// of Gauss-Jordan elimination, one block of pivots at a time). One workgroup
// inverts one matrix, which stays in device memory; the pivot block, the
// panel rows of a tile column and the old A_RP rows of a tile row are staged
// in LDS.
#include <hip/hip_runtime.h>

#include "device.h"

namespace ddmgnn {

namespace {

constexpr int GJ_THREADS = 256;
constexpr int GJ_W = 32;  // pivot block width
constexpr int GJ_T = 64;  // rows and columns of a tile of the trailing update (4 x 4 per thread)

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

struct GjShared {
    double D[GJ_W][GJ_W + 1];   // pivot block, then its inverse
    double F[GJ_T][GJ_W + 1];   // old A_RP rows of a tile row
    double R[GJ_W][GJ_T + 1];   // new A_PR columns of a tile column
    int bad;
};

// In-place inverse of the SPD matrix M (k x k, row stride ld); sets sh.bad when
// a pivot is not positive and finite (M is then not SPD and left undefined).
__device__ void gj_invert(double* __restrict__ M, int k, int64_t ld, GjShared& sh) {
    const int t = threadIdx.x;
    if (t == 0) sh.bad = 0;
    for (int pb = 0; pb < k; pb += GJ_W) {
        const int w = min(GJ_W, k - pb), pe = pb + w;
        // 1. The pivot block and its inverse (unblocked Gauss-Jordan in LDS).
        for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) {
            const int r = e / GJ_W, c = e % GJ_W;
            sh.D[r][c] = r < w && c < w ? M[(int64_t)(pb + r) * ld + pb + c] : 0.0;
        }
        __syncthreads();
        for (int q = 0; q < w; ++q) {
            const double dq = sh.D[q][q];
            if (!(dq > 0.0) || !isfinite(dq)) {
                if (t == 0) sh.bad = 1;
            }
            const double piv = 1.0 / dq;
            double nv[GJ_W * GJ_W / GJ_THREADS];
#pragma unroll
            for (int u = 0; u < GJ_W * GJ_W / GJ_THREADS; ++u) {
                const int e = t + u * GJ_THREADS, r = e / GJ_W, c = e % GJ_W;
                double v = sh.D[r][c];
                if (r == q && c == q) v = piv;
                else if (r == q) v = v * piv;
                else if (c == q) v = -v * piv;
                else v = fma(-sh.D[r][q] * piv, sh.D[q][c], v);
                nv[u] = v;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < GJ_W * GJ_W / GJ_THREADS; ++u) {
                const int e = t + u * GJ_THREADS;
                if (e / GJ_W < w && e % GJ_W < w) sh.D[e / GJ_W][e % GJ_W] = nv[u];
            }
            __syncthreads();
        }
        // 2. A_PR <- A_PP^{-1} A_PR, one column per thread.
        for (int j = t; j < k; j += GJ_THREADS) {
            if (j >= pb && j < pe) continue;
            double x[GJ_W];
#pragma unroll
            for (int r = 0; r < GJ_W; ++r) x[r] = r < w ? M[(int64_t)(pb + r) * ld + j] : 0.0;
            for (int r = 0; r < w; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < GJ_W; ++c) acc = fma(sh.D[r][c], x[c], acc);
                M[(int64_t)(pb + r) * ld + j] = acc;
            }
        }
        __syncthreads();
        // 3. Per tile row I (rows outside P): A_RR -= F A_PR(new) over the tile
        // columns outside P, with F the old A_RP rows; then A_RP <- -F A_PP^{-1}.
        const int ty = t / 16, tx = t % 16;
        for (int i0 = 0; i0 < k; i0 += GJ_T) {
            if (i0 >= pb && i0 + GJ_T <= pe) continue;  // the tile row lies inside P
            for (int e = t; e < GJ_T * GJ_W; e += GJ_THREADS) {
                const int r = e / GJ_W, c = e % GJ_W, i = i0 + r;
                sh.F[r][c] = i < k && (i < pb || i >= pe) && c < w ? M[(int64_t)i * ld + pb + c] : 0.0;
            }
            __syncthreads();
            for (int j0 = 0; j0 < k; j0 += GJ_T) {
                if (j0 >= pb && j0 + GJ_T <= pe) continue;
                for (int e = t; e < GJ_W * GJ_T; e += GJ_THREADS) {
                    const int r = e / GJ_T, c = e % GJ_T, j = j0 + c;
                    sh.R[r][c] = r < w && j < k && (j < pb || j >= pe) ? M[(int64_t)(pb + r) * ld + j] : 0.0;
                }
                __syncthreads();
                double acc[4][4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
                for (int p = 0; p < w; ++p) {
                    double f[4], g[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a) f[a] = sh.F[ty * 4 + a][p];
#pragma unroll
                    for (int b = 0; b < 4; ++b) g[b] = sh.R[p][tx * 4 + b];
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) acc[a][b] = fma(f[a], g[b], acc[a][b]);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int i = i0 + ty * 4 + a;
                    if (i >= k || (i >= pb && i < pe)) continue;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int j = j0 + tx * 4 + b;
                        if (j >= k || (j >= pb && j < pe)) continue;
                        M[(int64_t)i * ld + j] -= acc[a][b];
                    }
                }
                __syncthreads();
            }
            for (int e = t; e < GJ_T * GJ_W; e += GJ_THREADS) {
                const int r = e / GJ_W, c = e % GJ_W, i = i0 + r;
                if (i >= k || (i >= pb && i < pe) || c >= w) continue;
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < GJ_W; ++q) acc = fma(sh.F[r][q], sh.D[q][c], acc);
                M[(int64_t)i * ld + pb + c] = -acc;
            }
            __syncthreads();
        }
        // 4. A_PP <- A_PP^{-1}.
        for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) {
            const int r = e / GJ_W, c = e % GJ_W;
            if (r < w && c < w) M[(int64_t)(pb + r) * ld + pb + c] = sh.D[r][c];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(GJ_THREADS) void lu_invert_kernel(const int64_t* __restrict__ sub_ptr,
                                                                const int64_t* __restrict__ off,
                                                                double* __restrict__ inv, int* __restrict__ status) {
    __shared__ GjShared sh;
    const int i = blockIdx.x;
    const int k = (int)(sub_ptr[i + 1] - sub_ptr[i]);
    gj_invert(inv + off[i], k, (off[i + 1] - off[i]) / k, sh);
    if (threadIdx.x == 0 && sh.bad) atomicOr(status, 1);
}

// ---------------------------------------------------------------- coarse level
// A_0 = Z^T A Z (column i of Z is R_i^T D_i R_i 1, Sec. III.A step 1): row i of
// A_0 sums w_a A[g_a][m] w_b over the slots a of sub-mesh i, the nonzeros
// (g_a, m) of A and the slots b of node m (sub-mesh j = slot_sub[b]). One
// thread builds one row, in slot, nonzero and membership order, so the bits
// do not depend on scheduling.
__global__ __launch_bounds__(64) void coarse_assemble_kernel(const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ col,
                                                             const double* __restrict__ val,
                                                             const int32_t* __restrict__ sub_ptr,
                                                             const int32_t* __restrict__ sub_nodes,
                                                             const double* __restrict__ weights,
                                                             const int32_t* __restrict__ node_ptr,
                                                             const int32_t* __restrict__ node_slots,
                                                             const int32_t* __restrict__ slot_sub, int K,
                                                             double* __restrict__ a0) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= K) return;
    double* row = a0 + (size_t)i * K;
    for (int j = 0; j < K; ++j) row[j] = 0.0;
    for (int a = sub_ptr[i]; a < sub_ptr[i + 1]; ++a) {
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

__global__ __launch_bounds__(256) void diag_copy_kernel(const double* __restrict__ a, int K, double* __restrict__ d) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < K) d[i] = a[(size_t)i * K + i];
}

// Exact symmetry: both triangles take the mean of the two sums.
__global__ __launch_bounds__(256) void coarse_symmetrise_kernel(double* __restrict__ a0, int K) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)K * K) return;
    const int i = (int)(e / K), j = (int)(e % K);
    if (j <= i) return;
    const double m = 0.5 * (a0[(size_t)i * K + j] + a0[(size_t)j * K + i]);
    a0[(size_t)i * K + j] = m;
    a0[(size_t)j * K + i] = m;
}

// The coarse matrix is inverted with the same Gauss-Jordan steps as gj_invert,
// spread over the whole device: per pivot block, one workgroup inverts the
// block (into dinv), a grid updates the pivot rows, a grid of tiles updates
// the rest, and a grid writes the pivot columns and the pivot block.
// A pivot is accepted when it exceeds GJ_REL times the matrix's original
// diagonal entry (diag0; null: when it is positive): a singular or nearly
// singular A_0 is refused instead of inverted.
constexpr double GJ_REL = 1e-12;
__global__ __launch_bounds__(GJ_THREADS) void gj_pivot_kernel(const double* __restrict__ M, int k, int pb,
                                                              double* __restrict__ dinv, int* __restrict__ status,
                                                              const double* __restrict__ diag0) {
    __shared__ double D[GJ_W][GJ_W + 1];
    const int t = threadIdx.x, w = min(GJ_W, k - pb);
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) {
        const int r = e / GJ_W, c = e % GJ_W;
        D[r][c] = r < w && c < w ? M[(size_t)(pb + r) * k + pb + c] : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < w; ++q) {
        const double dq = D[q][q];
        const double floor = diag0 ? GJ_REL * fabs(diag0[pb + q]) : 0.0;
        if (t == 0 && (!(dq > floor) || !isfinite(dq))) atomicOr(status, 1);
        const double piv = 1.0 / dq;
        double nv[GJ_W * GJ_W / GJ_THREADS];
#pragma unroll
        for (int u = 0; u < GJ_W * GJ_W / GJ_THREADS; ++u) {
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
        for (int u = 0; u < GJ_W * GJ_W / GJ_THREADS; ++u) {
            const int e = t + u * GJ_THREADS;
            if (e / GJ_W < w && e % GJ_W < w) D[e / GJ_W][e % GJ_W] = nv[u];
        }
        __syncthreads();
    }
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) dinv[e] = D[e / GJ_W][e % GJ_W];
}

// A_PR(new) = dinv A_PR, one column per thread, into pr (GJ_W x k): the pivot
// rows of the matrix are replaced only after the tile update, which reads the
// old A_RP from the matrix and the new A_PR from pr.
__global__ __launch_bounds__(GJ_THREADS) void gj_rows_kernel(const double* __restrict__ M, int k, int pb,
                                                             const double* __restrict__ dinv, double* __restrict__ pr) {
    __shared__ double D[GJ_W][GJ_W + 1];
    const int t = threadIdx.x, w = min(GJ_W, k - pb);
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) D[e / GJ_W][e % GJ_W] = dinv[e];
    __syncthreads();
    const int j = blockIdx.x * GJ_THREADS + t;
    if (j >= k) return;
    double x[GJ_W];
#pragma unroll
    for (int r = 0; r < GJ_W; ++r) x[r] = r < w ? M[(size_t)(pb + r) * k + j] : 0.0;
    for (int r = 0; r < w; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < GJ_W; ++c) acc = fma(D[r][c], x[c], acc);
        pr[(size_t)r * k + j] = acc;
    }
}

// A_RR -= A_RP(old) A_PR(new) on one GJ_T x GJ_T tile per workgroup.
__global__ __launch_bounds__(GJ_THREADS) void gj_tiles_kernel(double* __restrict__ M, int k, int pb,
                                                              const double* __restrict__ pr) {
    __shared__ double F[GJ_T][GJ_W + 1];
    __shared__ double R[GJ_W][GJ_T + 1];
    const int t = threadIdx.x, w = min(GJ_W, k - pb), pe = pb + w;
    const int nt = (k + GJ_T - 1) / GJ_T;
    const int i0 = (blockIdx.x / nt) * GJ_T, j0 = (blockIdx.x % nt) * GJ_T;
    for (int e = t; e < GJ_T * GJ_W; e += GJ_THREADS) {
        const int r = e / GJ_W, c = e % GJ_W, i = i0 + r;
        F[r][c] = i < k && (i < pb || i >= pe) && c < w ? M[(size_t)i * k + pb + c] : 0.0;
    }
    for (int e = t; e < GJ_W * GJ_T; e += GJ_THREADS) {
        const int r = e / GJ_T, c = e % GJ_T, j = j0 + c;
        R[r][c] = r < w && j < k && (j < pb || j >= pe) ? pr[(size_t)r * k + j] : 0.0;
    }
    __syncthreads();
    const int ty = t / 16, tx = t % 16;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int p = 0; p < w; ++p) {
        double f[4], g[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) f[a] = F[ty * 4 + a][p];
#pragma unroll
        for (int b = 0; b < 4; ++b) g[b] = R[p][tx * 4 + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(f[a], g[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + ty * 4 + a;
        if (i >= k || (i >= pb && i < pe)) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + tx * 4 + b;
            if (j >= k || (j >= pb && j < pe)) continue;
            M[(size_t)i * k + j] -= acc[a][b];
        }
    }
}

// A_RP <- -A_RP(old) dinv (one row per thread), the pivot rows <- pr, and
// A_PP <- dinv.
__global__ __launch_bounds__(GJ_THREADS) void gj_cols_kernel(double* __restrict__ M, int k, int pb,
                                                             const double* __restrict__ dinv,
                                                             const double* __restrict__ pr) {
    __shared__ double D[GJ_W][GJ_W + 1];
    const int t = threadIdx.x, w = min(GJ_W, k - pb), pe = pb + w;
    for (int e = t; e < GJ_W * GJ_W; e += GJ_THREADS) D[e / GJ_W][e % GJ_W] = dinv[e];
    __syncthreads();
    const int i = blockIdx.x * GJ_THREADS + t;
    if (i >= k) return;
    if (i >= pb && i < pe) {  // pivot row: the new A_PR, and A_PP <- dinv
        const int r = i - pb;
        for (int j = 0; j < k; ++j) M[(size_t)i * k + j] = j >= pb && j < pe ? D[r][j - pb] : pr[(size_t)r * k + j];
        return;
    }
    double f[GJ_W];
#pragma unroll
    for (int c = 0; c < GJ_W; ++c) f[c] = c < w ? M[(size_t)i * k + pb + c] : 0.0;
    for (int c = 0; c < w; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < GJ_W; ++q) acc = fma(f[q], D[q][c], acc);
        M[(size_t)i * k + pb + c] = -acc;
    }
}

}  // namespace

hipError_t launch_coarse_setup(const int32_t* rowptr, const int32_t* col, const double* val, const int32_t* sub_ptr,
                               const int32_t* sub_nodes, const double* weights, const int32_t* node_ptr,
                               const int32_t* node_slots, const int32_t* slot_sub, int K, double* a0inv,
                               double* scratch, int* status, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(coarse_assemble_kernel, dim3((K + 63) / 64), dim3(64), 0, s, rowptr, col, val, sub_ptr,
                       sub_nodes, weights, node_ptr, node_slots, slot_sub, K, a0inv);
    const int64_t kk = (int64_t)K * K;
    hipLaunchKernelGGL(coarse_symmetrise_kernel, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, s, a0inv, K);
    double* dinv = scratch;                      // GJ_W x GJ_W
    double* pr = scratch + GJ_W * GJ_W;           // GJ_W x K
    double* diag0 = pr + (size_t)GJ_W * K;        // K: the diagonal of A_0
    hipLaunchKernelGGL(diag_copy_kernel, dim3((K + 255) / 256), dim3(256), 0, s, a0inv, K, diag0);
    const int nt = (K + GJ_T - 1) / GJ_T;
    const unsigned ncol = (unsigned)((K + GJ_THREADS - 1) / GJ_THREADS);
    for (int pb = 0; pb < K; pb += GJ_W) {
        hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(GJ_THREADS), 0, s, a0inv, K, pb, dinv, status, diag0);
        hipLaunchKernelGGL(gj_rows_kernel, dim3(ncol), dim3(GJ_THREADS), 0, s, a0inv, K, pb, dinv, pr);
        hipLaunchKernelGGL(gj_tiles_kernel, dim3((unsigned)(nt * nt)), dim3(GJ_THREADS), 0, s, a0inv, K, pb, pr);
        hipLaunchKernelGGL(gj_cols_kernel, dim3(ncol), dim3(GJ_THREADS), 0, s, a0inv, K, pb, dinv, pr);
    }
    return hipGetLastError();
}

size_t coarse_setup_scratch(int K) { return (size_t)GJ_W * GJ_W + (size_t)GJ_W * K + (size_t)K; }

hipError_t launch_lu_factor(const int32_t* rowptr, const int32_t* col, const double* val, const int64_t* sub_ptr,
                            const int32_t* sub_nodes, const int64_t* off, double* inv, int n_sub, int* status,
                            hipStream_t s) {
    if (n_sub <= 0) return hipSuccess;
    hipLaunchKernelGGL(lu_assemble_kernel, dim3(n_sub), dim3(GJ_THREADS), 0, s, rowptr, col, val, sub_ptr,
                       sub_nodes, off, inv);
    hipLaunchKernelGGL(lu_invert_kernel, dim3(n_sub), dim3(GJ_THREADS), 0, s, sub_ptr, off, inv, status);
    return hipGetLastError();
}

}  // namespace ddmgnn
