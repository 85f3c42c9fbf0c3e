// Host-side setup of a DDM-GNN problem. See setup.h.
#include "setup.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

namespace ddmgnn {

namespace {

// sum_p a[p] b[p] with four interleaved partial sums (a fixed order).
inline double dot4(const double* a, const double* b, int64_t len) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t p = 0;
    for (; p + 4 <= len; p += 4) {
        s0 += a[p] * b[p];
        s1 += a[p + 1] * b[p + 1];
        s2 += a[p + 2] * b[p + 2];
        s3 += a[p + 3] * b[p + 3];
    }
    for (; p < len; ++p) s0 += a[p] * b[p];
    return (s0 + s1) + (s2 + s3);
}

// ------------------------------------------------------------------ dense SPD inverse
// C[m x n] -= A[m x np] B[np x n] for one register tile (m <= 4, n <= 8), all
// row-major: A[r * lda + p], B[p * ldb + c], C[r * ldc + c]. Each entry sums p
// in increasing order. Compiled twice (AVX2 + FMA and the base instruction set)
// from one body; the first use picks the version the CPU runs.
typedef double v4d __attribute__((vector_size(32)));

__attribute__((always_inline)) inline v4d load4(const double* p) {
    v4d v;
    std::memcpy(&v, p, sizeof v);
    return v;
}

__attribute__((always_inline)) inline void tile_body(int m, int n, int np, const double* A, int64_t lda,
                                                     const double* B, int64_t ldb, double* C, int64_t ldc) {
    if (m == 4 && n == 8) {
        v4d c[4][2] = {};
        const double *a0 = A, *a1 = A + lda, *a2 = A + 2 * lda, *a3 = A + 3 * lda;
        for (int p = 0; p < np; ++p) {
            const v4d b0 = load4(B + p * ldb), b1 = load4(B + p * ldb + 4);
            const double x0 = a0[p], x1 = a1[p], x2 = a2[p], x3 = a3[p];
            c[0][0] += x0 * b0; c[0][1] += x0 * b1;
            c[1][0] += x1 * b0; c[1][1] += x1 * b1;
            c[2][0] += x2 * b0; c[2][1] += x2 * b1;
            c[3][0] += x3 * b0; c[3][1] += x3 * b1;
        }
        for (int r = 0; r < 4; ++r)
            for (int h = 0; h < 2; ++h) {
                const v4d v = load4(C + r * ldc + 4 * h) - c[r][h];
                std::memcpy(C + r * ldc + 4 * h, &v, sizeof v);
            }
        return;
    }
    double acc[4][8] = {};
    for (int p = 0; p < np; ++p)
        for (int r = 0; r < m; ++r)
            for (int q = 0; q < n; ++q) acc[r][q] += A[r * lda + p] * B[p * ldb + q];
    for (int r = 0; r < m; ++r)
        for (int q = 0; q < n; ++q) C[r * ldc + q] -= acc[r][q];
}

__attribute__((target("avx2,fma"))) void tile_avx2(int m, int n, int np, const double* A, int64_t lda,
                                                   const double* B, int64_t ldb, double* C, int64_t ldc) {
    tile_body(m, n, np, A, lda, B, ldb, C, ldc);
}

void tile_base(int m, int n, int np, const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
               int64_t ldc) {
    tile_body(m, n, np, A, lda, B, ldb, C, ldc);
}

using TileFn = void (*)(int, int, int, const double*, int64_t, const double*, int64_t, double*, int64_t);

TileFn tile_fn() {
    static const TileFn f = [] {
        __builtin_cpu_init();
        return __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma") ? &tile_avx2 : &tile_base;
    }();
    return f;
}

// inv = A^{-1} for the symmetric positive definite K x K matrix a (row-major),
// in three blocked steps of K^3/6 multiply-adds each:
//   1. A = L L^T (right-looking, panels of 64; the trailing update in tiles),
//   2. Y = L^{-1} (block rows; the part left of the diagonal block in tiles),
//   3. A^{-1} = Y^T Y (lower triangle in tiles, mirrored).
// With `parallel`, the tiles of each step are spread over host threads (each
// tile on one thread, so the result does not depend on the thread count).
// Returns false when a pivot is not positive.
bool dense_cholesky(const std::vector<double>& a, int32_t K, std::vector<double>& inv, bool parallel = true) {
    auto pfor = [&](int64_t n, auto&& f) {
        if (parallel)
            parallel_for(n, f);
        else
            for (int64_t i = 0; i < n; ++i) f(i);
    };
    const TileFn tile = tile_fn();
    constexpr int32_t B = 64;
    std::vector<double> L(a);
    auto at = [&](int64_t i, int64_t j) -> double& { return L[(size_t)i * K + j]; };
    std::vector<double> panel;
    // 1. Cholesky; only the lower triangle of L is read (the tiles of the
    // trailing update also write entries right of the diagonal, never read).
    for (int32_t kb = 0; kb < K; kb += B) {
        const int32_t ke = std::min(K, kb + B), w = ke - kb, m = K - ke;
        for (int32_t j = kb; j < ke; ++j) {
            const double dsum = at(j, j) - dot4(&at(j, kb), &at(j, kb), j - kb);
            if (!(dsum > 0.0) || !std::isfinite(dsum)) return false;
            at(j, j) = std::sqrt(dsum);
            for (int32_t i = j + 1; i < ke; ++i) at(i, j) = (at(i, j) - dot4(&at(i, kb), &at(j, kb), j - kb)) / at(j, j);
        }
        pfor(m, [&](int64_t t) {
            const int64_t i = ke + t;
            for (int32_t j = kb; j < ke; ++j) at(i, j) = (at(i, j) - dot4(&at(i, kb), &at(j, kb), j - kb)) / at(j, j);
        });
        // panel transposed: panel[p * m + j] = L[ke + j][kb + p]
        panel.assign((size_t)w * m, 0.0);
        for (int32_t j = 0; j < m; ++j)
            for (int32_t p = 0; p < w; ++p) panel[(size_t)p * m + j] = at(ke + j, kb + p);
        pfor((m + 3) / 4, [&](int64_t t) {
            const int32_t i0 = (int32_t)t * 4, rows = std::min(4, m - i0);
            for (int32_t j0 = 0; j0 < i0 + rows; j0 += 8)
                tile(rows, std::min(8, m - j0), w, &at(ke + i0, kb), K, &panel[j0], m, &at(ke + i0, ke + j0), K);
        });
    }
    // 2. Y = L^{-1}, lower triangular, zeros above the diagonal. Rows of block
    // [ib, ie): first C = -L[I][0:ib] Y[0:ib][0:ib] (Y[p][c] = 0 for p < c, so
    // column tile c0 starts at p = c0), then forward substitution within the block.
    std::vector<double> Y((size_t)K * K, 0.0);
    auto y = [&](int64_t i, int64_t j) -> double& { return Y[(size_t)i * K + j]; };
    for (int32_t ib = 0; ib < K; ib += B) {
        const int32_t ie = std::min(K, ib + B), w = ie - ib;
        pfor((ib + 7) / 8, [&](int64_t t) {
            const int32_t c0 = (int32_t)t * 8, cols = std::min(8, ib - c0);
            for (int32_t r0 = 0; r0 < w; r0 += 4)
                tile(std::min(4, w - r0), cols, ib - c0, &at(ib + r0, c0), K, &y(c0, c0), K, &y(ib + r0, c0), K);
        });
        for (int32_t i = ib; i < ie; ++i) {
            const double dinv = 1.0 / at(i, i);
            double* yi = &y(i, 0);
            for (int32_t q = ib; q < i; ++q) {
                const double l = at(i, q);
                const double* yq = &y(q, 0);
                for (int32_t c = 0; c <= q; ++c) yi[c] -= l * yq[c];
            }
            yi[i] += 1.0;
            for (int32_t c = 0; c <= i; ++c) yi[c] *= dinv;
        }
    }
    // 3. A^{-1} = Y^T Y. With Yt = -Y^T (upper triangular, in L's storage), the
    // tile C -= Yt Y gives X[a][b] = sum_p Y[p][a] Y[p][b]; rows a0.. start at
    // p = a0 (earlier terms are zero).
    for (int64_t i = 0; i < K; ++i)
        for (int64_t j = 0; j < K; ++j) at(i, j) = j >= i ? -y(j, i) : 0.0;
    inv.assign((size_t)K * K, 0.0);
    pfor((K + 3) / 4, [&](int64_t t) {
        const int32_t a0 = (int32_t)t * 4, rows = std::min(4, K - a0);
        for (int32_t b0 = 0; b0 < a0 + rows; b0 += 8)
            tile(rows, std::min(8, K - b0), K - a0, &at(a0, a0), K, &y(a0, b0), K, &inv[(size_t)a0 * K + b0], K);
    });
    // mirror the lower triangle (exactly symmetric inverse)
    for (int64_t i = 0; i < K; ++i)
        for (int64_t j = 0; j < i; ++j) inv[(size_t)j * K + i] = inv[(size_t)i * K + j];
    return true;
}

}  // namespace


namespace {

// Sorted, de-duplicated mesh adjacency (nodes sharing a triangle edge).
void mesh_adjacency(int64_t n, int64_t nt, const int32_t* tri, std::vector<int64_t>& ptr,
                    std::vector<int32_t>& adj) {
    // Triangles scatter both directions of their edges into per-node ranges on
    // host threads (any order), then each node's range is sorted and made unique,
    // which fixes the result whatever the scatter order.
    constexpr int64_t CH = 1 << 15;
    std::vector<std::atomic<int64_t>> cnt((size_t)n + 1);
    parallel_for((n + CH) / CH, [&](int64_t c) {
        for (int64_t i = c * CH; i < std::min(n + 1, (c + 1) * CH); ++i) cnt[i].store(0, std::memory_order_relaxed);
    });
    parallel_for((nt + CH - 1) / CH, [&](int64_t c) {
        for (int64_t t = c * CH; t < std::min(nt, (c + 1) * CH); ++t)
            for (int i = 0; i < 3; ++i) cnt[tri[3 * t + i] + 1].fetch_add(2, std::memory_order_relaxed);
    });
    std::vector<int64_t> start((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + cnt[i + 1].load(std::memory_order_relaxed);
    std::vector<int32_t> tmp((size_t)start[n]);
    parallel_for((n + CH - 1) / CH, [&](int64_t c) {
        for (int64_t i = c * CH; i < std::min(n, (c + 1) * CH); ++i) cnt[i].store(start[i], std::memory_order_relaxed);
    });
    parallel_for((nt + CH - 1) / CH, [&](int64_t c) {
        for (int64_t t = c * CH; t < std::min(nt, (c + 1) * CH); ++t)
            for (int i = 0; i < 3; ++i) {
                const int32_t a = tri[3 * t + i], b = tri[3 * t + (i + 1) % 3];
                tmp[cnt[a].fetch_add(1, std::memory_order_relaxed)] = b;
                tmp[cnt[b].fetch_add(1, std::memory_order_relaxed)] = a;
            }
    });
    std::vector<int64_t> uniq((size_t)n + 1, 0);
    parallel_for((n + CH - 1) / CH, [&](int64_t c) {
        for (int64_t i = c * CH; i < std::min(n, (c + 1) * CH); ++i) {
            auto b = tmp.begin() + start[i], e = tmp.begin() + start[i + 1];
            std::sort(b, e);
            uniq[i + 1] = std::unique(b, e) - b;
        }
    });
    ptr.assign((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + uniq[i + 1];
    adj.resize((size_t)ptr[n]);
    parallel_for((n + CH - 1) / CH, [&](int64_t c) {
        for (int64_t i = c * CH; i < std::min(n, (c + 1) * CH); ++i)
            std::copy(tmp.begin() + start[i], tmp.begin() + start[i] + (ptr[i + 1] - ptr[i]), adj.begin() + ptr[i]);
    });
}

}  // namespace

// The message of the lowest index i in [0, n) for which check(i) fails
// (returns a message), or nullptr: chunks of indices on host threads, so the
// result is that of a serial loop.
template <class F>
const char* first_failure(int64_t n, F&& check) {
    constexpr int64_t CH = 1 << 15;
    const int64_t nc = (n + CH - 1) / CH;
    std::vector<const char*> msg((size_t)nc, nullptr);
    parallel_for(nc, [&](int64_t c) {
        for (int64_t i = c * CH; i < std::min(n, (c + 1) * CH); ++i)
            if (const char* m = check(i)) {
                msg[(size_t)c] = m;
                return;
            }
    });
    for (const char* m : msg)
        if (m) return m;
    return nullptr;
}

std::string validate(const ddmgnn_problem_desc& d) {
    const int64_t n = d.n_nodes;
    if (n <= 0) return "n_nodes must be positive";
    if (n >= (1ll << 31)) return "n_nodes must fit int32";
    if (!d.xy || !d.tri || !d.dirichlet || !d.a_rowptr || !d.a_col || !d.a_val || !d.b || !d.u0 ||
        !d.sub_ptr || !d.sub_nodes || !d.weights)
        return "null pointer in problem descriptor";
    if (d.n_tri <= 0) return "n_tri must be positive";
    if (const char* m = first_failure(3 * d.n_tri, [&](int64_t t) -> const char* {
            return d.tri[t] < 0 || d.tri[t] >= n ? "triangle node id out of range" : nullptr;
        }))
        return m;
    if (const char* m = first_failure(n, [&](int64_t i) -> const char* {
            if (d.dirichlet[i] > 1) return "dirichlet flags must be 0 or 1";
            if (!std::isfinite(d.xy[2 * i]) || !std::isfinite(d.xy[2 * i + 1])) return "non-finite coordinate";
            if (!std::isfinite(d.b[i]) || !std::isfinite(d.u0[i])) return "non-finite b or u0";
            return nullptr;
        }))
        return m;
    if (d.a_rowptr[0] != 0) return "a_rowptr[0] must be 0";
    if (const char* m = first_failure(n, [&](int64_t i) -> const char* {
            int32_t s = d.a_rowptr[i], e = d.a_rowptr[i + 1];
            if (e < s) return "a_rowptr must be non-decreasing";
            bool diag = false;
            for (int32_t k = s; k < e; ++k) {
                int32_t c = d.a_col[k];
                if (c < 0 || c >= n) return "column index out of range";
                if (k > s && c <= d.a_col[k - 1]) return "columns must be strictly ascending in each row";
                if (!std::isfinite(d.a_val[k])) return "non-finite matrix value";
                if (c == i) diag = true;
                if (d.dirichlet[i] && c != i) return "Dirichlet rows must be identity rows";
                if (d.dirichlet[i] && d.a_val[k] != 1.0) return "Dirichlet rows must be identity rows";
                if (!d.dirichlet[i] && d.dirichlet[c]) return "free rows must not couple to Dirichlet nodes";
            }
            return diag ? nullptr : "missing diagonal entry";
        }))
        return m;
    // Symmetry: for every (i, c, v) the entry (c, i) exists with the same value
    // (the rows are valid by now).
    if (const char* m = first_failure(n, [&](int64_t i) -> const char* {
            for (int32_t k = d.a_rowptr[i]; k < d.a_rowptr[i + 1]; ++k) {
                int32_t c = d.a_col[k];
                const int32_t* b = d.a_col + d.a_rowptr[c];
                const int32_t* e = d.a_col + d.a_rowptr[c + 1];
                const int32_t* it = std::lower_bound(b, e, (int32_t)i);
                if (it == e || *it != i || d.a_val[it - d.a_col] != d.a_val[k]) return "matrix is not symmetric";
            }
            return nullptr;
        }))
        return m;
    if (d.n_sub <= 0) return "n_sub must be positive";
    if (d.sub_ptr[0] != 0) return "sub_ptr[0] must be 0";
    std::vector<double> wsum(n, 0.0);
    std::vector<int32_t> cover(n, 0);
    for (int32_t s = 0; s < d.n_sub; ++s) {
        int64_t b = d.sub_ptr[s], e = d.sub_ptr[s + 1];
        if (e <= b) return "empty sub-mesh";
        if (e - b > kMaxSubNodesAny) return "sub-mesh larger than the supported maximum (16384 nodes)";
        for (int64_t k = b; k < e; ++k) {
            int32_t v = d.sub_nodes[k];
            if (v < 0 || v >= n) return "sub_nodes id out of range";
            if (k > b && v <= d.sub_nodes[k - 1]) return "sub_nodes must be strictly ascending per sub-mesh";
            double w = d.weights[k];
            if (!std::isfinite(w) || w < 0) return "weights must be finite and non-negative";
            wsum[v] += w;
            cover[v] += 1;
        }
    }
    if (d.sub_ptr[d.n_sub] >= (1ll << 31)) return "total sub-mesh size must fit int32";
    for (int64_t i = 0; i < n; ++i) {
        if (!cover[i]) return "node not covered by any sub-mesh";
        if (d.dirichlet[i] && wsum[i] != 0.0) return "weights must be 0 at Dirichlet nodes";
        if (!d.dirichlet[i] && std::fabs(wsum[i] - 1.0) > 1e-12) return "weights are not a partition of unity";
    }
    return "";
}

void expand_overlap(int64_t n, int64_t nt, const int32_t* tri, const int32_t* part, int32_t n_part,
                    int32_t delta, std::vector<int64_t>& sub_ptr, std::vector<int32_t>& sub_nodes) {
    std::vector<int64_t> aptr;
    std::vector<int32_t> adj;
    mesh_adjacency(n, nt, tri, aptr, adj);
    std::vector<std::vector<int32_t>> core(n_part);
    for (int64_t i = 0; i < n; ++i) core[part[i]].push_back((int32_t)i);
    std::vector<int32_t> mark(n, -1);
    sub_ptr.assign(1, 0);
    sub_nodes.clear();
    for (int32_t p = 0; p < n_part; ++p) {
        std::vector<int32_t> members = core[p], front = core[p];
        for (int32_t v : members) mark[v] = p;
        for (int32_t layer = 0; layer < delta; ++layer) {
            std::vector<int32_t> next;
            for (int32_t v : front)
                for (int64_t e = aptr[v]; e < aptr[v + 1]; ++e)
                    if (mark[adj[e]] != p) {
                        mark[adj[e]] = p;
                        next.push_back(adj[e]);
                    }
            members.insert(members.end(), next.begin(), next.end());
            front.swap(next);
        }
        std::sort(members.begin(), members.end());
        sub_nodes.insert(sub_nodes.end(), members.begin(), members.end());
        sub_ptr.push_back((int64_t)sub_nodes.size());
    }
}

void build_local_graphs(const ddmgnn_problem_desc& d, HostSetup& s) {
    const int64_t n = d.n_nodes;
    const int32_t K = d.n_sub;
    s.n = n;
    s.nnz = d.a_rowptr[n];
    s.K = K;
    s.sk = d.sub_ptr[K];
    s.sub_ptr.assign(d.sub_ptr, d.sub_ptr + K + 1);
    std::vector<int64_t> aptr;
    std::vector<int32_t> adj;
    mesh_adjacency(n, d.n_tri, d.tri, aptr, adj);

    // Local DSS graphs. The local index of a node is its rank in the sorted
    // sub-mesh list, and a receiver's global neighbours are sorted, so walking
    // them yields senders in ascending local order. Sub-meshes are independent:
    // first count each slot's in-edges, then fill them.
    auto local_of = [&](int64_t b, int64_t e, int32_t g) -> int32_t {
        const int32_t* first = d.sub_nodes + b;
        const int32_t* last = d.sub_nodes + e;
        const int32_t* it = std::lower_bound(first, last, g);
        return (it != last && *it == g) ? (int32_t)(it - first) : -1;
    };
    s.edge_ptr.assign(s.sk + 1, 0);
    s.slot_sub.assign(s.sk, 0);
    parallel_for(K, [&](int64_t i) {
        const int64_t b = d.sub_ptr[i], e = d.sub_ptr[i + 1];
        for (int64_t k = b; k < e; ++k) {
            const int32_t j = d.sub_nodes[k];
            s.slot_sub[k] = (int32_t)i;
            int64_t c = 0;
            if (!d.dirichlet[j])
                for (int64_t a = aptr[j]; a < aptr[j + 1]; ++a) c += local_of(b, e, adj[a]) >= 0;
            s.edge_ptr[k + 1] = c;
        }
    });
    for (int64_t k = 0; k < s.sk; ++k) s.edge_ptr[k + 1] += s.edge_ptr[k];
    s.n_edges = s.edge_ptr[s.sk];
    s.edge_src.assign(s.n_edges, 0);
    s.max_k = 0;
    for (int32_t i = 0; i < K; ++i) s.max_k = std::max<int32_t>(s.max_k, (int32_t)(d.sub_ptr[i + 1] - d.sub_ptr[i]));

    // Membership lists: slots of every node, in increasing slot order.
    s.node_ptr.assign(n + 1, 0);
    for (int64_t k = 0; k < s.sk; ++k) s.node_ptr[d.sub_nodes[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) s.node_ptr[i + 1] += s.node_ptr[i];
    s.node_slots.assign(s.sk, 0);
    {
        std::vector<int64_t> pos(s.node_ptr.begin(), s.node_ptr.end() - 1);
        for (int64_t k = 0; k < s.sk; ++k) s.node_slots[pos[d.sub_nodes[k]]++] = (int32_t)k;
    }
    s.work_order.resize(K);
    std::iota(s.work_order.begin(), s.work_order.end(), 0);
    std::stable_sort(s.work_order.begin(), s.work_order.end(), [&](int32_t a, int32_t b) {
        return d.sub_ptr[a + 1] - d.sub_ptr[a] > d.sub_ptr[b + 1] - d.sub_ptr[b];
    });

    // Per sub-mesh: senders, tile order, centred split coordinates and edge lengths.
    s.tnode.assign(s.sk, 0);
    s.xyhl.assign(4 * s.sk, 0);
    s.xyc.assign(2 * s.sk, 0.0);
    s.erec.assign(s.n_edges, 0u);
    s.edge_nd.assign(s.n_edges, 0.0f);
    parallel_for(K, [&](int64_t i) {
        const int64_t b = d.sub_ptr[i], e = d.sub_ptr[i + 1];
        const int32_t k = (int32_t)(e - b);
        for (int64_t q = b; q < e; ++q) {
            const int32_t j = d.sub_nodes[q];
            if (d.dirichlet[j]) continue;
            int64_t t = s.edge_ptr[q];
            for (int64_t a = aptr[j]; a < aptr[j + 1]; ++a) {
                const int32_t l = local_of(b, e, adj[a]);
                if (l >= 0) s.edge_src[t++] = (uint16_t)l;
            }
        }
        std::vector<int32_t> ord(k);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
            return s.edge_ptr[b + x + 1] - s.edge_ptr[b + x] > s.edge_ptr[b + y + 1] - s.edge_ptr[b + y];
        });
        for (int32_t q = 0; q < k; ++q) s.tnode[b + q] = (uint16_t)ord[q];
        double cx = 0, cy = 0;
        for (int64_t q = b; q < e; ++q) {
            cx += d.xy[2 * d.sub_nodes[q]];
            cy += d.xy[2 * d.sub_nodes[q] + 1];
        }
        cx /= k;
        cy /= k;
        for (int64_t q = b; q < e; ++q) {
            const double x = d.xy[2 * d.sub_nodes[q]] - cx, y = d.xy[2 * d.sub_nodes[q] + 1] - cy;
            s.xyc[2 * q] = x;
            s.xyc[2 * q + 1] = y;
            const uint16_t xh = bf16_rne_bits((float)x), yh = bf16_rne_bits((float)y);
            s.xyhl[4 * q + 0] = xh;
            s.xyhl[4 * q + 1] = bf16_rne_bits((float)(x - bf16_bits_float(xh)));
            s.xyhl[4 * q + 2] = yh;
            s.xyhl[4 * q + 3] = bf16_rne_bits((float)(y - bf16_bits_float(yh)));
        }
        for (int64_t q = b; q < e; ++q) {
            const int32_t j = d.sub_nodes[q];
            for (int64_t t = s.edge_ptr[q]; t < s.edge_ptr[q + 1]; ++t) {
                const int32_t l = d.sub_nodes[b + s.edge_src[t]];
                const double dx = d.xy[2 * l] - d.xy[2 * j], dy = d.xy[2 * l + 1] - d.xy[2 * j + 1];
                s.edge_nd[t] = (float)std::sqrt(dx * dx + dy * dy);
                const _Float16 hnd = (_Float16)s.edge_nd[t];
                uint16_t bits;
                std::memcpy(&bits, &hnd, 2);
                s.erec[t] = (uint32_t)s.edge_src[t] | ((uint32_t)bits << 16);
            }
        }
    });
    s.max_edges_sub = 0;
    for (int32_t i = 0; i < K; ++i)
        s.max_edges_sub = std::max<int64_t>(s.max_edges_sub, s.edge_ptr[d.sub_ptr[i + 1]] - s.edge_ptr[d.sub_ptr[i]]);
}

std::string local_inverse(const ddmgnn_problem_desc& d, int32_t i, std::vector<double>& inv, bool parallel) {
    const int64_t b = d.sub_ptr[i], e = d.sub_ptr[i + 1];
    const int32_t k = (int32_t)(e - b);
    std::vector<double> a((size_t)k * k, 0.0);
    for (int32_t j = 0; j < k; ++j) {
        const int32_t g = d.sub_nodes[b + j];
        for (int32_t t = d.a_rowptr[g]; t < d.a_rowptr[g + 1]; ++t) {
            const int32_t c = d.a_col[t];
            const int32_t* first = d.sub_nodes + b;
            const int32_t* it = std::lower_bound(first, d.sub_nodes + e, c);
            if (it != d.sub_nodes + e && *it == c) a[(size_t)j * k + (it - first)] = d.a_val[t];
        }
    }
    if (!dense_cholesky(a, k, inv, parallel)) return "NOT_SPD";
    return "";
}

std::string build_local_inverses(const ddmgnn_problem_desc& d, std::vector<double>& inv, std::vector<int64_t>& off) {
    const int32_t K = d.n_sub;
    off.assign(K + 1, 0);
    for (int32_t i = 0; i < K; ++i) {
        const int64_t k = d.sub_ptr[i + 1] - d.sub_ptr[i];
        off[i + 1] = off[i] + k * lu_ld(k);
    }
    inv.assign((size_t)off[K], 0.0);
    std::atomic<int32_t> bad{-1};
    parallel_for(K, [&](int64_t i) {
        std::vector<double> m;
        if (!local_inverse(d, (int32_t)i, m, false).empty()) {
            bad.store((int32_t)i);
            return;
        }
        const int64_t k = d.sub_ptr[i + 1] - d.sub_ptr[i], ld = lu_ld(k);
        for (int64_t r = 0; r < k; ++r)
            std::memcpy(&inv[(size_t)(off[i] + r * ld)], &m[(size_t)(r * k)], k * sizeof(double));
    });
    return bad.load() >= 0 ? "NOT_SPD" : "";
}

std::string build_setup(const ddmgnn_problem_desc& d, HostSetup& s, bool coarse) {
    build_local_graphs(d, s);
    if (!coarse) return "";
    const int64_t n = d.n_nodes;
    const int32_t K = d.n_sub;

    // Coarse operator: column j of Z is D_j on sub-mesh j; A_0[i][j] = Z_i^T A Z_j.
    // For each j, v = A Z_j is accumulated on the rows it touches, then
    // scattered to A_0[sub(slot)][j] through the membership lists.
    s.a0.assign((size_t)K * K, 0.0);
    std::vector<double> v(n, 0.0);
    std::vector<char> touched(n, 0);
    std::vector<int32_t> rows;
    for (int32_t j = 0; j < K; ++j) {
        rows.clear();
        for (int64_t k = d.sub_ptr[j]; k < d.sub_ptr[j + 1]; ++k) {
            int32_t m = d.sub_nodes[k];
            double w = d.weights[k];
            if (w == 0.0) continue;
            // column m of A equals row m (symmetric)
            for (int32_t e = d.a_rowptr[m]; e < d.a_rowptr[m + 1]; ++e) {
                int32_t r = d.a_col[e];
                if (!touched[r]) { touched[r] = 1; rows.push_back(r); }
                v[r] += d.a_val[e] * w;
            }
        }
        for (int32_t r : rows) {
            for (int64_t q = s.node_ptr[r]; q < s.node_ptr[r + 1]; ++q) {
                int32_t slot = s.node_slots[q];
                s.a0[(size_t)s.slot_sub[slot] * K + j] += d.weights[slot] * v[r];
            }
            v[r] = 0.0;
            touched[r] = 0;
        }
    }
    // Symmetrise exactly (both triangles hold the same value up to rounding order).
    for (int32_t i = 0; i < K; ++i)
        for (int32_t j = i + 1; j < K; ++j) {
            double a = 0.5 * (s.a0[(size_t)i * K + j] + s.a0[(size_t)j * K + i]);
            s.a0[(size_t)i * K + j] = s.a0[(size_t)j * K + i] = a;
        }
    // Cholesky A_0 = L L^T (lower, row-major), then A_0^{-1} = L^{-T} L^{-1}.
    if (!dense_cholesky(s.a0, K, s.a0inv)) return "NOT_SPD";
    return "";
}

}  // namespace ddmgnn
