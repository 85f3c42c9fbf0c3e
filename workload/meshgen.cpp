// Seeded synthetic workload generator: star-shaped polygon, Delaunay mesh,
// P1 finite-element assembly of the Poisson-Dirichlet problem, recursive
// coordinate bisection into non-overlapping parts.
//
// This file is input generation only. It builds the problem the solver is
// given (mesh, A, b, partition into cores), as the problem statement of the
// paper sets it up (Sec. II, eqs. (1)-(2); dataset recipe of Sec. IV.A with a
// star polygon in place of the Bezier/GMSH domain and bisection in place of
// METIS). It contains none of the preconditioner or Krylov arithmetic.
//
// Determinism: all randomness comes from splitmix64 counters; the Delaunay
// predicates are exact (integer coordinates, 128-bit incircle), so the same
// seed yields the same bytes on every machine.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

// ---------------------------------------------------------------- RNG
static inline uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline double u01(uint64_t& s) {  // [0,1) with 53 bits
    return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
}
static inline double usym(uint64_t& s) { return 2.0 * u01(s) - 1.0; }  // [-1,1)

// ---------------------------------------------------------------- geometry
struct Poly {
    std::vector<double> x, y;  // vertices, counter-clockwise
    bool inside(double px, double py) const {
        bool in = false;
        size_t n = x.size();
        for (size_t i = 0, j = n - 1; i < n; j = i++) {
            if (((y[i] > py) != (y[j] > py)) &&
                (px < (x[j] - x[i]) * (py - y[i]) / (y[j] - y[i]) + x[i]))
                in = !in;
        }
        return in;
    }
    double dist(double px, double py) const {
        double best = 1e300;
        size_t n = x.size();
        for (size_t i = 0; i < n; ++i) {
            size_t j = (i + 1) % n;
            double ex = x[j] - x[i], ey = y[j] - y[i];
            double t = ((px - x[i]) * ex + (py - y[i]) * ey) / (ex * ex + ey * ey);
            t = std::min(1.0, std::max(0.0, t));
            double dx = px - (x[i] + t * ex), dy = py - (y[i] + t * ey);
            best = std::min(best, std::sqrt(dx * dx + dy * dy));
        }
        return best;
    }
    double area() const {
        double a = 0;
        size_t n = x.size();
        for (size_t i = 0; i < n; ++i) {
            size_t j = (i + 1) % n;
            a += x[i] * y[j] - x[j] * y[i];
        }
        return 0.5 * a;
    }
};

static inline uint64_t morton_key(int64_t x, int64_t y) {
    // coordinates shifted to be non-negative, 31 bits each
    uint64_t ux = (uint64_t)(x + (1ll << 30)), uy = (uint64_t)(y + (1ll << 30));
    uint64_t k = 0;
    for (int b = 0; b < 31; ++b) {
        k |= ((ux >> b) & 1ull) << (2 * b);
        k |= ((uy >> b) & 1ull) << (2 * b + 1);
    }
    return k;
}

// ---------------------------------------------------------------- Delaunay
// Incremental Bowyer-Watson with exact predicates on integer coordinates.
struct Delaunay {
    std::vector<int64_t> X, Y;  // point coordinates (grid units)
    struct Tri {
        int v[3];
        int n[3];  // n[i]: neighbour across the edge opposite v[i]
    };
    std::vector<Tri> T;
    std::vector<uint32_t> stamp;
    std::vector<char> alive;
    std::vector<int> free_slots;
    uint32_t cur_stamp = 0;
    int last = 0;

    int64_t orient(int a, int b, int c) const {
        return (X[b] - X[a]) * (Y[c] - Y[a]) - (Y[b] - Y[a]) * (X[c] - X[a]);
    }
    // > 0 when d lies strictly inside the circumcircle of counter-clockwise abc
    bool incircle(int a, int b, int c, int d) const {
        __int128 adx = X[a] - X[d], ady = Y[a] - Y[d];
        __int128 bdx = X[b] - X[d], bdy = Y[b] - Y[d];
        __int128 cdx = X[c] - X[d], cdy = Y[c] - Y[d];
        __int128 det = (adx * adx + ady * ady) * (bdx * cdy - cdx * bdy) +
                       (bdx * bdx + bdy * bdy) * (cdx * ady - adx * cdy) +
                       (cdx * cdx + cdy * cdy) * (adx * bdy - bdx * ady);
        return det > 0;
    }
    int new_tri() {
        if (!free_slots.empty()) {
            int t = free_slots.back();
            free_slots.pop_back();
            alive[t] = 1;
            return t;
        }
        T.push_back(Tri{});
        stamp.push_back(0);
        alive.push_back(1);
        return (int)T.size() - 1;
    }
    int locate(int p) {
        int t = last;
        unsigned rot = 0;
        for (;;) {
            const Tri& tr = T[t];
            int moved = -1;
            for (int k = 0; k < 3; ++k) {
                int i = (int)((k + rot) % 3);
                int a = tr.v[(i + 1) % 3], b = tr.v[(i + 2) % 3];
                if (orient(a, b, p) < 0) { moved = tr.n[i]; break; }
            }
            if (moved < 0) return t;
            t = moved;
            ++rot;
        }
    }
    void insert(int p) {
        int t0 = locate(p);
        ++cur_stamp;
        std::vector<int> cav{t0};
        stamp[t0] = cur_stamp;
        for (size_t q = 0; q < cav.size(); ++q) {
            const Tri& c = T[cav[q]];
            for (int i = 0; i < 3; ++i) {
                int nb = c.n[i];
                if (nb < 0 || stamp[nb] == cur_stamp) continue;
                const Tri& o = T[nb];
                if (incircle(o.v[0], o.v[1], o.v[2], p)) {
                    stamp[nb] = cur_stamp;
                    cav.push_back(nb);
                }
            }
        }
        struct BE { int a, b, outer, outer_slot; };
        std::vector<BE> be;
        for (int c : cav) {
            const Tri& tr = T[c];
            for (int i = 0; i < 3; ++i) {
                int nb = tr.n[i];
                if (nb >= 0 && stamp[nb] == cur_stamp) continue;
                int slot = -1;
                if (nb >= 0)
                    for (int j = 0; j < 3; ++j)
                        if (T[nb].n[j] == c) slot = j;
                be.push_back({tr.v[(i + 1) % 3], tr.v[(i + 2) % 3], nb, slot});
            }
        }
        for (int c : cav) { alive[c] = 0; free_slots.push_back(c); }
        std::vector<int> nt(be.size());
        for (size_t k = 0; k < be.size(); ++k) {
            int t = new_tri();
            nt[k] = t;
            T[t].v[0] = be[k].a; T[t].v[1] = be[k].b; T[t].v[2] = p;
            T[t].n[2] = be[k].outer;
            if (be[k].outer >= 0) T[be[k].outer].n[be[k].outer_slot] = t;
            stamp[t] = 0;
        }
        for (size_t k = 0; k < be.size(); ++k) {
            for (size_t m = 0; m < be.size(); ++m) {
                if (be[m].a == be[k].b) T[nt[k]].n[0] = nt[m];
                if (be[m].b == be[k].a) T[nt[k]].n[1] = nt[m];
            }
        }
        last = nt[0];
    }
};

struct Mesh {
    std::vector<double> xy;
    std::vector<int32_t> tri;
    std::vector<uint8_t> dirichlet;
    std::vector<double> poly;  // polygon vertices (x0,y0,x1,y1,...)
    double R = 0;
};

}  // namespace

extern "C" {

// Generate a mesh. h = element size, unit = h/1024 grid. Returns a handle.
void* wl_mesh_generate(uint64_t seed, int64_t target_nodes, double h) {
    Mesh* M = new Mesh;
    uint64_t rs = seed * 0x2545F4914F6CDD1Dull + 0x1234567ull;
    // Star polygon: 8..12 vertices, angular jitter 1/4 slot, radius jitter 0.3.
    int nv = 8 + (int)(splitmix64(rs) % 5ull);
    std::vector<double> ang(nv), rad(nv);
    for (int k = 0; k < nv; ++k) {
        ang[k] = 2.0 * M_PI * (k + 0.25 * usym(rs)) / nv;
        rad[k] = 1.0 + 0.3 * usym(rs);
    }
    Poly unit;
    for (int k = 0; k < nv; ++k) {
        unit.x.push_back(rad[k] * std::cos(ang[k]));
        unit.y.push_back(rad[k] * std::sin(ang[k]));
    }
    double a1 = unit.area();
    // Lattice density: one node per (sqrt(3)/2) h^2.
    double R = h * std::sqrt((double)target_nodes * (std::sqrt(3.0) / 2.0) / a1);
    M->R = R;
    Poly P;
    for (int k = 0; k < nv; ++k) {
        P.x.push_back(R * unit.x[k]);
        P.y.push_back(R * unit.y[k]);
        M->poly.push_back(P.x.back());
        M->poly.push_back(P.y.back());
    }
    const double unitlen = h / 1024.0;
    std::vector<std::pair<int64_t, int64_t>> pts;
    auto snap = [&](double x, double y) {
        pts.push_back({(int64_t)std::llround(x / unitlen), (int64_t)std::llround(y / unitlen)});
    };
    // Boundary subdivision at spacing ~h.
    for (int k = 0; k < nv; ++k) {
        int j = (k + 1) % nv;
        double ex = P.x[j] - P.x[k], ey = P.y[j] - P.y[k];
        double L = std::sqrt(ex * ex + ey * ey);
        int ns = std::max(1, (int)std::llround(L / h));
        for (int s = 0; s < ns; ++s) snap(P.x[k] + ex * s / ns, P.y[k] + ey * s / ns);
    }
    std::vector<std::pair<int64_t, int64_t>> bpts(pts.begin(), pts.end());
    std::sort(bpts.begin(), bpts.end());
    // Jittered triangular lattice, kept at >= 0.5h from the boundary.
    double xmin = *std::min_element(P.x.begin(), P.x.end());
    double xmax = *std::max_element(P.x.begin(), P.x.end());
    double ymin = *std::min_element(P.y.begin(), P.y.end());
    double ymax = *std::max_element(P.y.begin(), P.y.end());
    double dy = h * std::sqrt(3.0) / 2.0;
    int64_t j0 = (int64_t)std::floor(ymin / dy) - 1, j1 = (int64_t)std::ceil(ymax / dy) + 1;
    int64_t i0 = (int64_t)std::floor(xmin / h) - 2, i1 = (int64_t)std::ceil(xmax / h) + 2;
    for (int64_t j = j0; j <= j1; ++j) {
        for (int64_t i = i0; i <= i1; ++i) {
            double x = i * h + ((j & 1) ? 0.5 * h : 0.0) + 0.2 * h * usym(rs);
            double y = j * dy + 0.2 * h * usym(rs);
            if (!P.inside(x, y)) continue;
            if (P.dist(x, y) < 0.5 * h) continue;
            snap(x, y);
        }
    }
    // Deduplicate, then order along a Morton curve (insertion order and final numbering).
    std::sort(pts.begin(), pts.end());
    pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
    std::vector<uint64_t> key(pts.size());
    for (size_t i = 0; i < pts.size(); ++i) key[i] = morton_key(pts[i].first, pts[i].second);
    std::vector<int> ord(pts.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) {
        return key[a] != key[b] ? key[a] < key[b] : pts[a] < pts[b];
    });
    Delaunay D;
    int np = (int)pts.size();
    D.X.resize(np + 3);
    D.Y.resize(np + 3);
    for (int k = 0; k < np; ++k) { D.X[k] = pts[ord[k]].first; D.Y[k] = pts[ord[k]].second; }
    const int64_t S = 1ll << 24;
    D.X[np] = -S; D.Y[np] = -S;
    D.X[np + 1] = S; D.Y[np + 1] = -S;
    D.X[np + 2] = 0; D.Y[np + 2] = S;
    int t0 = D.new_tri();
    D.T[t0].v[0] = np; D.T[t0].v[1] = np + 1; D.T[t0].v[2] = np + 2;
    D.T[t0].n[0] = D.T[t0].n[1] = D.T[t0].n[2] = -1;
    D.last = t0;
    for (int k = 0; k < np; ++k) D.insert(k);
    std::vector<char> on_poly(np, 0);
    for (int k = 0; k < np; ++k)
        on_poly[k] = std::binary_search(bpts.begin(), bpts.end(), pts[ord[k]]) ? 1 : 0;
    // Largest angle of a triangle, in degrees.
    auto max_angle = [&](int a, int b, int c) {
        int v[3] = {a, b, c};
        double best = 0;
        for (int i = 0; i < 3; ++i) {
            double ux = (double)(D.X[v[(i + 1) % 3]] - D.X[v[i]]), uy = (double)(D.Y[v[(i + 1) % 3]] - D.Y[v[i]]);
            double wx = (double)(D.X[v[(i + 2) % 3]] - D.X[v[i]]), wy = (double)(D.Y[v[(i + 2) % 3]] - D.Y[v[i]]);
            double cs = (ux * wx + uy * wy) / std::sqrt((ux * ux + uy * uy) * (wx * wx + wy * wy));
            best = std::max(best, std::acos(std::max(-1.0, std::min(1.0, cs))) * 180.0 / M_PI);
        }
        return best;
    };
    // Keep triangles of real points whose centroid is inside the polygon.
    int nt = (int)D.T.size();
    std::vector<char> keep(nt, 0);
    for (int t = 0; t < nt; ++t) {
        if (!D.alive[t]) continue;
        const auto& tr = D.T[t];
        if (tr.v[0] >= np || tr.v[1] >= np || tr.v[2] >= np) continue;
        double cx = (D.X[tr.v[0]] + D.X[tr.v[1]] + D.X[tr.v[2]]) * unitlen / 3.0;
        double cy = (D.Y[tr.v[0]] + D.Y[tr.v[1]] + D.Y[tr.v[2]]) * unitlen / 3.0;
        if (D.orient(tr.v[0], tr.v[1], tr.v[2]) <= 0) continue;
        // Near-flat triangles spanned by three boundary points (snapping makes
        // subdivision points of one polygon edge slightly non-collinear).
        if (on_poly[tr.v[0]] && on_poly[tr.v[1]] && on_poly[tr.v[2]] &&
            max_angle(tr.v[0], tr.v[1], tr.v[2]) > 150.0)
            continue;
        keep[t] = P.inside(cx, cy) ? 1 : 0;
    }
    // Largest edge-connected component of kept triangles.
    std::vector<int> comp(nt, -1);
    int best_c = -1;
    size_t best_sz = 0;
    for (int t = 0, c = 0; t < nt; ++t) {
        if (!keep[t] || comp[t] >= 0) continue;
        std::vector<int> st{t};
        comp[t] = c;
        size_t sz = 0;
        while (!st.empty()) {
            int u = st.back();
            st.pop_back();
            ++sz;
            for (int i = 0; i < 3; ++i) {
                int nb = D.T[u].n[i];
                if (nb >= 0 && keep[nb] && comp[nb] < 0) { comp[nb] = c; st.push_back(nb); }
            }
        }
        if (sz > best_sz) { best_sz = sz; best_c = c; }
        ++c;
    }
    std::vector<int> newid(np, -1);
    std::vector<char> bnd(np, 0);
    for (int t = 0; t < nt; ++t) {
        if (!keep[t] || comp[t] != best_c) continue;
        for (int i = 0; i < 3; ++i) {
            newid[D.T[t].v[i]] = 0;
            int nb = D.T[t].n[i];
            bool inner = nb >= 0 && keep[nb] && comp[nb] == best_c;
            if (!inner) {
                bnd[D.T[t].v[(i + 1) % 3]] = 1;
                bnd[D.T[t].v[(i + 2) % 3]] = 1;
            }
        }
    }
    int nn = 0;
    for (int k = 0; k < np; ++k)
        if (newid[k] == 0) newid[k] = nn++;
    M->xy.resize(2 * (size_t)nn);
    M->dirichlet.resize(nn);
    for (int k = 0; k < np; ++k) {
        if (newid[k] < 0) continue;
        M->xy[2 * newid[k]] = D.X[k] * unitlen;
        M->xy[2 * newid[k] + 1] = D.Y[k] * unitlen;
        M->dirichlet[newid[k]] = bnd[k];
    }
    for (int t = 0; t < nt; ++t) {
        if (!keep[t] || comp[t] != best_c) continue;
        for (int i = 0; i < 3; ++i) M->tri.push_back(newid[D.T[t].v[i]]);
    }
    // Order triangles by their lowest vertex for locality (deterministic).
    size_t ntri = M->tri.size() / 3;
    std::vector<int> to(ntri);
    std::iota(to.begin(), to.end(), 0);
    auto tkey = [&](int t) {
        const int32_t* v = &M->tri[3 * (size_t)t];
        return std::min(v[0], std::min(v[1], v[2]));
    };
    std::stable_sort(to.begin(), to.end(), [&](int a, int b) { return tkey(a) < tkey(b); });
    std::vector<int32_t> tri2(M->tri.size());
    for (size_t k = 0; k < ntri; ++k)
        for (int i = 0; i < 3; ++i) tri2[3 * k + i] = M->tri[3 * (size_t)to[k] + i];
    M->tri.swap(tri2);
    return M;
}

void wl_mesh_sizes(void* hdl, int64_t* n_nodes, int64_t* n_tri, int64_t* n_poly, double* R) {
    Mesh* M = (Mesh*)hdl;
    *n_nodes = (int64_t)M->dirichlet.size();
    *n_tri = (int64_t)(M->tri.size() / 3);
    *n_poly = (int64_t)(M->poly.size() / 2);
    *R = M->R;
}

void wl_mesh_copy(void* hdl, double* xy, int32_t* tri, uint8_t* dirichlet, double* poly) {
    Mesh* M = (Mesh*)hdl;
    std::memcpy(xy, M->xy.data(), M->xy.size() * sizeof(double));
    std::memcpy(tri, M->tri.data(), M->tri.size() * sizeof(int32_t));
    std::memcpy(dirichlet, M->dirichlet.data(), M->dirichlet.size());
    std::memcpy(poly, M->poly.data(), M->poly.size() * sizeof(double));
}

void wl_mesh_free(void* hdl) { delete (Mesh*)hdl; }

// P1 Galerkin assembly of -Laplace u = f with Dirichlet data g (eqs. (1)-(2)).
// f_mid[3t+k] is f at the midpoint of the edge of triangle t opposite its local
// vertex k (edge-midpoint quadrature, exact for quadratics). With eliminate=1
// the Dirichlet rows/columns are eliminated symmetrically (identity rows,
// b_B = g_B, b_I -= A_IB g_B) and the dropped entries removed; with
// eliminate=0 the unconstrained stiffness matrix and load are returned.
// Output arrays have capacity `cap` entries; returns nnz, or -1 if cap is short.
int64_t wl_assemble(int64_t n, const double* xy, int64_t nt, const int32_t* tri,
                    const uint8_t* dirichlet, const double* f_mid, const double* g,
                    int eliminate, int32_t* rowptr, int32_t* col, double* val,
                    double* b, int64_t cap) {
    std::vector<std::vector<int32_t>> adj(n);
    for (int64_t t = 0; t < nt; ++t)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) adj[tri[3 * t + i]].push_back(tri[3 * t + j]);
    std::vector<int64_t> rp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        auto& a = adj[i];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        if (a.empty()) a.push_back((int32_t)i);
        rp[i + 1] = rp[i] + (int64_t)a.size();
    }
    std::vector<int32_t> c(rp[n]);
    std::vector<double> v(rp[n], 0.0);
    for (int64_t i = 0; i < n; ++i) std::copy(adj[i].begin(), adj[i].end(), c.begin() + rp[i]);
    std::vector<double> bb(n, 0.0);
    auto add = [&](int32_t r, int32_t cc, double x) {
        auto it = std::lower_bound(c.begin() + rp[r], c.begin() + rp[r + 1], cc);
        v[it - c.begin()] += x;
    };
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* vv = &tri[3 * t];
        double x[3], y[3];
        for (int i = 0; i < 3; ++i) { x[i] = xy[2 * vv[i]]; y[i] = xy[2 * vv[i] + 1]; }
        double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
        double area = 0.5 * std::fabs(det);
        double be[3], ga[3];
        for (int i = 0; i < 3; ++i) {
            int j = (i + 1) % 3, k = (i + 2) % 3;
            be[i] = y[j] - y[k];
            ga[i] = x[k] - x[j];
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                add(vv[i], vv[j], (be[i] * be[j] + ga[i] * ga[j]) / (4.0 * area));
        for (int i = 0; i < 3; ++i) {
            int j = (i + 1) % 3, k = (i + 2) % 3;
            bb[vv[i]] += area / 6.0 * (f_mid[3 * t + j] + f_mid[3 * t + k]);
        }
    }
    int64_t nnz = 0;
    rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (eliminate && dirichlet[i]) {
            if (nnz + 1 > cap) return -1;
            col[nnz] = (int32_t)i;
            val[nnz] = 1.0;
            ++nnz;
            b[i] = g[i];
        } else {
            double bi = bb[i];
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                int32_t j = c[e];
                if (eliminate && dirichlet[j]) { bi -= v[e] * g[j]; continue; }
                if (nnz + 1 > cap) return -1;
                col[nnz] = j;
                val[nnz] = v[e];
                ++nnz;
            }
            b[i] = bi;
        }
        rowptr[i + 1] = (int32_t)nnz;
    }
    return nnz;
}

// Recursive coordinate bisection into n_parts non-overlapping parts (stands in
// for METIS, Sec. IV.A). Each split cuts along the principal axis of the node
// coordinates; the node share of the first half is proportional to its part
// count, scaled by (1 + jitter*U[-1,1]) to make uneven parts. Ties in the
// projection are broken by node id.
void wl_partition_rcb(int64_t n, const double* xy, int32_t n_parts, double jitter,
                      uint64_t seed, int32_t* part) {
    std::vector<int32_t> ids(n);
    std::iota(ids.begin(), ids.end(), 0);
    struct Job { int64_t lo, hi; int32_t k, first; };
    std::vector<Job> st{{0, n, n_parts, 0}};
    uint64_t split_counter = 0;
    std::vector<std::pair<double, int32_t>> key;
    while (!st.empty()) {
        Job jb = st.back();
        st.pop_back();
        if (jb.k <= 1) {
            for (int64_t i = jb.lo; i < jb.hi; ++i) part[ids[i]] = jb.first;
            continue;
        }
        int64_t m = jb.hi - jb.lo;
        double mx = 0, my = 0;
        for (int64_t i = jb.lo; i < jb.hi; ++i) { mx += xy[2 * ids[i]]; my += xy[2 * ids[i] + 1]; }
        mx /= (double)m; my /= (double)m;
        double sxx = 0, syy = 0, sxy = 0;
        for (int64_t i = jb.lo; i < jb.hi; ++i) {
            double dx = xy[2 * ids[i]] - mx, dy = xy[2 * ids[i] + 1] - my;
            sxx += dx * dx; syy += dy * dy; sxy += dx * dy;
        }
        // Principal eigenvector of [[sxx, sxy], [sxy, syy]].
        double tr = sxx + syy, dt = sxx * syy - sxy * sxy;
        double lam = 0.5 * tr + std::sqrt(std::max(0.0, 0.25 * tr * tr - dt));
        double ax, ay;
        if (std::fabs(sxy) > 1e-300) { ax = lam - syy; ay = sxy; }
        else if (sxx >= syy) { ax = 1; ay = 0; }
        else { ax = 0; ay = 1; }
        double nrm = std::sqrt(ax * ax + ay * ay);
        ax /= nrm; ay /= nrm;
        key.resize(m);
        for (int64_t i = 0; i < m; ++i) {
            int32_t id = ids[jb.lo + i];
            key[i] = {xy[2 * id] * ax + xy[2 * id + 1] * ay, id};
        }
        std::sort(key.begin(), key.end());
        for (int64_t i = 0; i < m; ++i) ids[jb.lo + i] = key[i].second;
        int32_t k1 = jb.k / 2, k2 = jb.k - k1;
        uint64_t s = seed ^ (0xD1B54A32D192ED03ull * (++split_counter));
        double frac = (double)k1 / jb.k * (1.0 + jitter * usym(s));
        frac = std::min(0.9, std::max(0.1, frac));
        int64_t n1 = std::llround(frac * (double)m);
        n1 = std::max<int64_t>(k1, std::min<int64_t>(m - k2, n1));
        st.push_back({jb.lo + n1, jb.hi, k2, jb.first + k1});
        st.push_back({jb.lo, jb.lo + n1, k1, jb.first});
    }
}

}  // extern "C"
