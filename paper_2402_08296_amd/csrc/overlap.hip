// Overlapping decomposition on the device (Sec. II.A; overlap of Sec. IV.A):
// sub-mesh i is part i grown by delta layers of mesh adjacency (nodes sharing
// a triangle), with the partition-of-unity weights 1/multiplicity at free
// nodes and 0 at Dirichlet nodes. The same sets, in ascending node order, as
// the host helper (expand_overlap, pou weights).
//
// Every node keeps the sorted set of the parts whose sub-meshes hold it. A
// round of growth replaces a node's set by the union of its own and those of
// the nodes of its triangles (reading the previous round's sets, so the
// result does not depend on scheduling); delta rounds grow every part by
// delta layers at once. The sub-mesh lists are then counted, filled and
// sorted per part.
#include <hip/hip_runtime.h>

#include "device.h"

namespace ddmgnn {

namespace {

constexpr int OV_THREADS = 256;
constexpr int SCAN_THREADS = 1024;

__global__ __launch_bounds__(OV_THREADS) void ov_check_kernel(const int32_t* __restrict__ tri, int64_t n3,
                                                              const int32_t* __restrict__ part, int64_t n,
                                                              int32_t n_part, int* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (i < n3 && (tri[i] < 0 || tri[i] >= n)) atomicOr(status, 1);
    if (i < n && (part[i] < 0 || part[i] >= n_part)) atomicOr(status, 2);
}

// Triangles of each node: counts, then (after the scan) the lists in any order.
__global__ __launch_bounds__(OV_THREADS) void ov_tri_count_kernel(const int32_t* __restrict__ tri, int64_t n3,
                                                                  int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (i < n3) atomicAdd(&cnt[tri[i]], 1);
}
__global__ __launch_bounds__(OV_THREADS) void ov_tri_fill_kernel(const int32_t* __restrict__ tri, int64_t n3,
                                                                 const int64_t* __restrict__ ptr,
                                                                 int32_t* __restrict__ cur,
                                                                 int32_t* __restrict__ list) {
    const int64_t i = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (i >= n3) return;
    const int32_t v = tri[i];
    list[ptr[v] + atomicAdd(&cur[v], 1)] = (int32_t)(i / 3);
}

// Exclusive scan of n counts into ptr[0..n] (one workgroup: each thread sums a
// contiguous chunk, the chunk sums are scanned in LDS, then the chunks are
// written).
__global__ __launch_bounds__(SCAN_THREADS) void ov_scan_kernel(const int32_t* __restrict__ cnt, int64_t n,
                                                               int64_t* __restrict__ ptr) {
    __shared__ int64_t part_sum[SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t chunk = (n + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b = min((int64_t)t * chunk, n), e = min(b + chunk, n);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += cnt[i];
    part_sum[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int i = 0; i < SCAN_THREADS; ++i) {
            const int64_t v = part_sum[i];
            part_sum[i] = acc;
            acc += v;
        }
        ptr[n] = acc;
    }
    __syncthreads();
    int64_t acc = part_sum[t];
    for (int64_t i = b; i < e; ++i) {
        ptr[i] = acc;
        acc += cnt[i];
    }
}

// Inserts p into the ascending set s[0..m) of capacity OV_CAP; returns the new
// size, or OV_CAP + 1 on overflow.
__device__ inline int set_insert(int32_t (&s)[OV_CAP], int m, int32_t p) {
    int pos = 0;
    while (pos < m && s[pos] < p) ++pos;
    if (pos < m && s[pos] == p) return m;
    if (m == OV_CAP) return OV_CAP + 1;
    for (int q = m; q > pos; --q) s[q] = s[q - 1];
    s[pos] = p;
    return m + 1;
}

__global__ __launch_bounds__(OV_THREADS) void ov_init_kernel(const int32_t* __restrict__ part, int64_t n,
                                                             int32_t* __restrict__ sets, uint8_t* __restrict__ sz) {
    const int64_t v = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (v >= n) return;
    sets[v * OV_CAP] = part[v];
    sz[v] = 1;
}

// One layer: next(v) = sets(v) united with the sets of the nodes of v's triangles.
__global__ __launch_bounds__(OV_THREADS) void ov_grow_kernel(const int32_t* __restrict__ tri,
                                                             const int64_t* __restrict__ tptr,
                                                             const int32_t* __restrict__ tlist, int64_t n,
                                                             const int32_t* __restrict__ sets,
                                                             const uint8_t* __restrict__ sz,
                                                             int32_t* __restrict__ nsets, uint8_t* __restrict__ nsz,
                                                             int* __restrict__ status) {
    const int64_t v = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (v >= n) return;
    int32_t s[OV_CAP];
    int m = sz[v];
    for (int q = 0; q < m; ++q) s[q] = sets[v * OV_CAP + q];
    for (int64_t e = tptr[v]; e < tptr[v + 1] && m <= OV_CAP; ++e) {
        const int64_t t = tlist[e];
        for (int c = 0; c < 3 && m <= OV_CAP; ++c) {
            const int32_t u = tri[3 * t + c];
            if (u == v) continue;
            for (int q = 0; q < sz[u] && m <= OV_CAP; ++q) m = set_insert(s, m, sets[(int64_t)u * OV_CAP + q]);
        }
    }
    if (m > OV_CAP) {
        atomicOr(status, 4);
        m = OV_CAP;
    }
    for (int q = 0; q < m; ++q) nsets[v * OV_CAP + q] = s[q];
    nsz[v] = (uint8_t)m;
}

__global__ __launch_bounds__(OV_THREADS) void ov_part_count_kernel(const int32_t* __restrict__ sets,
                                                                   const uint8_t* __restrict__ sz, int64_t n,
                                                                   int32_t* __restrict__ cnt) {
    const int64_t v = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (v >= n) return;
    for (int q = 0; q < sz[v]; ++q) atomicAdd(&cnt[sets[v * OV_CAP + q]], 1);
}

// The sub-mesh lists, each in any order.
__global__ __launch_bounds__(OV_THREADS) void ov_part_fill_kernel(const int32_t* __restrict__ sets,
                                                                  const uint8_t* __restrict__ sz, int64_t n,
                                                                  const int64_t* __restrict__ sptr,
                                                                  int32_t* __restrict__ cur,
                                                                  int32_t* __restrict__ nodes) {
    const int64_t v = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (v >= n) return;
    for (int q = 0; q < sz[v]; ++q) {
        const int32_t p = sets[v * OV_CAP + q];
        nodes[sptr[p] + atomicAdd(&cur[p], 1)] = (int32_t)v;
    }
}

// Ascending order of each sub-mesh's list (bitonic sort in LDS, one workgroup
// per sub-mesh of at most OV_SORT_MAX nodes).
__global__ __launch_bounds__(OV_THREADS) void ov_sort_kernel(const int64_t* __restrict__ sptr,
                                                             int32_t* __restrict__ nodes) {
    __shared__ int32_t key[OV_SORT_MAX];
    const int64_t b = sptr[blockIdx.x];
    const int k = (int)(sptr[blockIdx.x + 1] - b);
    int np = 1;
    while (np < k) np <<= 1;
    for (int i = threadIdx.x; i < np; i += OV_THREADS) key[i] = i < k ? nodes[b + i] : INT32_MAX;
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < np; i += OV_THREADS) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const int32_t a = key[i], c = key[j];
                    if ((a > c) == up) {
                        key[i] = c;
                        key[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < k; i += OV_THREADS) nodes[b + i] = key[i];
}

// Weights aligned with the sorted lists: 1/multiplicity at free nodes, 0 at
// Dirichlet nodes (the multiplicity of a node is the size of its part set).
__global__ __launch_bounds__(OV_THREADS) void ov_weights_kernel(const int32_t* __restrict__ nodes, int64_t sk,
                                                                const uint8_t* __restrict__ sz,
                                                                const uint8_t* __restrict__ dirichlet,
                                                                double* __restrict__ weights) {
    const int64_t i = (int64_t)blockIdx.x * OV_THREADS + threadIdx.x;
    if (i >= sk) return;
    const int32_t v = nodes[i];
    weights[i] = dirichlet[v] ? 0.0 : 1.0 / (double)sz[v];
}

unsigned grid(int64_t n) { return (unsigned)((n + OV_THREADS - 1) / OV_THREADS); }

}  // namespace

hipError_t ov_check(const int32_t* tri, int64_t n_tri, const int32_t* part, int64_t n, int32_t n_part, int* status,
                    hipStream_t s) {
    hipLaunchKernelGGL(ov_check_kernel, dim3(grid(std::max<int64_t>(3 * n_tri, n))), dim3(OV_THREADS), 0, s, tri,
                       3 * n_tri, part, n, n_part, status);
    return hipGetLastError();
}

hipError_t ov_grow(const int32_t* tri, int64_t n_tri, const int32_t* part, int64_t n, int32_t delta,
                   int32_t* tri_cnt, int64_t* tri_ptr, int32_t* tri_list, int32_t* sets0, int32_t* sets1,
                   uint8_t* sz0, uint8_t* sz1, int32_t** sets_out, uint8_t** sz_out, int* status, hipStream_t s) {
    const int64_t n3 = 3 * n_tri;
    hipLaunchKernelGGL(ov_tri_count_kernel, dim3(grid(n3)), dim3(OV_THREADS), 0, s, tri, n3, tri_cnt);
    hipLaunchKernelGGL(ov_scan_kernel, dim3(1), dim3(SCAN_THREADS), 0, s, tri_cnt, n, tri_ptr);
    hipError_t e = hipMemsetAsync(tri_cnt, 0, (size_t)n * sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ov_tri_fill_kernel, dim3(grid(n3)), dim3(OV_THREADS), 0, s, tri, n3, tri_ptr, tri_cnt,
                       tri_list);
    hipLaunchKernelGGL(ov_init_kernel, dim3(grid(n)), dim3(OV_THREADS), 0, s, part, n, sets0, sz0);
    int32_t* a = sets0;
    int32_t* b = sets1;
    uint8_t* za = sz0;
    uint8_t* zb = sz1;
    for (int32_t l = 0; l < delta; ++l) {
        hipLaunchKernelGGL(ov_grow_kernel, dim3(grid(n)), dim3(OV_THREADS), 0, s, tri, tri_ptr, tri_list, n, a, za,
                           b, zb, status);
        std::swap(a, b);
        std::swap(za, zb);
    }
    *sets_out = a;
    *sz_out = za;
    return hipGetLastError();
}

hipError_t ov_count(const int32_t* sets, const uint8_t* sz, int64_t n, int32_t n_part, int32_t* part_cnt,
                    int64_t* sub_ptr, hipStream_t s) {
    hipLaunchKernelGGL(ov_part_count_kernel, dim3(grid(n)), dim3(OV_THREADS), 0, s, sets, sz, n, part_cnt);
    hipLaunchKernelGGL(ov_scan_kernel, dim3(1), dim3(SCAN_THREADS), 0, s, part_cnt, (int64_t)n_part, sub_ptr);
    return hipGetLastError();
}

hipError_t ov_fill(const int32_t* sets, const uint8_t* sz, int64_t n, const uint8_t* dirichlet, int32_t n_part,
                   const int64_t* sub_ptr, int64_t sk, int32_t* part_cur, int32_t* nodes, double* weights,
                   hipStream_t s) {
    hipLaunchKernelGGL(ov_part_fill_kernel, dim3(grid(n)), dim3(OV_THREADS), 0, s, sets, sz, n, sub_ptr, part_cur,
                       nodes);
    hipLaunchKernelGGL(ov_sort_kernel, dim3(n_part), dim3(OV_THREADS), 0, s, sub_ptr, nodes);
    hipLaunchKernelGGL(ov_weights_kernel, dim3(grid(sk)), dim3(OV_THREADS), 0, s, nodes, sk, sz, dirichlet, weights);
    return hipGetLastError();
}

}  // namespace ddmgnn
