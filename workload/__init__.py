"""Seeded synthetic workload generator (input generation only).

Builds the problems the solver is given: a random star-shaped polygon, a
Delaunay triangle mesh of it, the P1 finite-element system A u = b of the
Poisson-Dirichlet problem (paper Sec. II, eqs. (1)-(2)), a non-overlapping
partition of the nodes into K parts, and seeded Xavier-uniform DSS weights.

It stands in for the paper's dataset recipe (Sec. IV.A: Bezier domains meshed
by GMSH, METIS parts of about 1000 nodes, quadratic f and g): the domain is a
star polygon (8-12 vertices, radius jitter 0.3), f is a sum of four Gaussians
with amplitudes in [-10, 10], g is the paper's random quadratic. Larger N grows
the radius at fixed element size, as the paper does.

Nothing here computes any part of the preconditioner or the Krylov method; both
the CPU oracle and the GPU library consume these arrays unchanged.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "meshgen.cpp")
_LIB = os.path.join(_HERE, "libworkload.so")

# Element size (power of two so mesh coordinates are exact binary fractions).
ELEMENT_SIZE = 2.0 ** -5


def build() -> str:
    """Compile the generator into workload/libworkload.so (always rebuilds)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        c_p = ctypes.c_void_p
        lib.wl_mesh_generate.restype = c_p
        lib.wl_mesh_generate.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double]
        lib.wl_mesh_sizes.argtypes = [c_p] + [ctypes.POINTER(ctypes.c_int64)] * 3 + [ctypes.POINTER(ctypes.c_double)]
        lib.wl_mesh_copy.argtypes = [c_p] * 5
        lib.wl_mesh_free.argtypes = [c_p]
        lib.wl_assemble.restype = ctypes.c_int64
        lib.wl_assemble.argtypes = [ctypes.c_int64, c_p, ctypes.c_int64, c_p, c_p, c_p, c_p,
                                    ctypes.c_int, c_p, c_p, c_p, c_p, ctypes.c_int64]
        lib.wl_partition_rcb.argtypes = [ctypes.c_int64, c_p, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_uint64, c_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Mesh:
    xy: np.ndarray          # [N, 2] float64
    tri: np.ndarray         # [T, 3] int32, counter-clockwise
    dirichlet: np.ndarray   # [N] uint8, 1 on the mesh boundary
    poly: np.ndarray        # [V, 2] polygon vertices
    R: float                # polygon scale

    @property
    def n(self) -> int:
        return self.xy.shape[0]


def make_mesh(seed: int, target_nodes: int, h: float = ELEMENT_SIZE) -> Mesh:
    lib = _load()
    hdl = lib.wl_mesh_generate(ctypes.c_uint64(seed), int(target_nodes), float(h))
    n, t, v = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    R = ctypes.c_double()
    lib.wl_mesh_sizes(hdl, ctypes.byref(n), ctypes.byref(t), ctypes.byref(v), ctypes.byref(R))
    xy = np.empty((n.value, 2), np.float64)
    tri = np.empty((t.value, 3), np.int32)
    dr = np.empty(n.value, np.uint8)
    poly = np.empty((v.value, 2), np.float64)
    lib.wl_mesh_copy(hdl, _ptr(xy), _ptr(tri), _ptr(dr), _ptr(poly))
    lib.wl_mesh_free(hdl)
    return Mesh(xy, tri, dr, poly, R.value)


def edge_midpoints(mesh: Mesh) -> np.ndarray:
    """[T, 3, 2] midpoint of the edge opposite each local vertex."""
    p = mesh.xy[mesh.tri]  # [T,3,2]
    return 0.5 * (p[:, [1, 2, 0]] + p[:, [2, 0, 1]])


@dataclass
class CSR:
    rowptr: np.ndarray  # int32 [N+1]
    col: np.ndarray     # int32 [nnz], ascending within a row
    val: np.ndarray     # float64 [nnz]

    @property
    def n(self) -> int:
        return self.rowptr.shape[0] - 1

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def assemble(mesh: Mesh, f_mid: np.ndarray, g: np.ndarray, eliminate: bool = True):
    """P1 stiffness and load (see meshgen.cpp). Returns (CSR, b)."""
    lib = _load()
    n, nt = mesh.n, mesh.tri.shape[0]
    cap = n + 6 * nt
    rowptr = np.empty(n + 1, np.int32)
    col = np.empty(cap, np.int32)
    val = np.empty(cap, np.float64)
    b = np.empty(n, np.float64)
    f_mid = np.ascontiguousarray(f_mid, np.float64).reshape(nt, 3)
    g = np.ascontiguousarray(g, np.float64)
    nnz = lib.wl_assemble(n, _ptr(mesh.xy), nt, _ptr(mesh.tri), _ptr(mesh.dirichlet), _ptr(f_mid),
                          _ptr(g), int(eliminate), _ptr(rowptr), _ptr(col), _ptr(val), _ptr(b), cap)
    if nnz < 0:
        raise RuntimeError("assembly capacity exceeded")
    return CSR(rowptr, col[:nnz].copy(), val[:nnz].copy()), b


def partition_rcb(xy: np.ndarray, n_parts: int, jitter: float, seed: int) -> np.ndarray:
    lib = _load()
    xy = np.ascontiguousarray(xy, np.float64)
    part = np.empty(xy.shape[0], np.int32)
    lib.wl_partition_rcb(xy.shape[0], _ptr(xy), int(n_parts), float(jitter), ctypes.c_uint64(seed),
                         _ptr(part))
    return part


# ----------------------------------------------------------------- f and g
@dataclass
class Forcing:
    amp: np.ndarray    # [4]
    mu: np.ndarray     # [4, 2]
    sigma: np.ndarray  # [4]
    gq: np.ndarray     # [6] quadratic coefficients r4..r9 of g in (x/R, y/R)
    R: float

    def f(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        out = np.zeros_like(x)
        for a, (mx, my), s in zip(self.amp, self.mu, self.sigma):
            out += a * np.exp(-((x - mx) ** 2 + (y - my) ** 2) / (2.0 * s * s))
        return out

    def g(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        xs, ys = x / self.R, y / self.R
        r4, r5, r6, r7, r8, r9 = self.gq
        return r4 * xs * xs + r5 * ys * ys + r6 * xs * ys + r7 * xs + r8 * ys + r9


def _point_in_poly(poly: np.ndarray, x: float, y: float) -> bool:
    inside = False
    n = poly.shape[0]
    j = n - 1
    for i in range(n):
        xi, yi = poly[i]
        xj, yj = poly[j]
        if (yi > y) != (yj > y) and x < (xj - xi) * (y - yi) / (yj - yi) + xi:
            inside = not inside
        j = i
    return inside


def make_forcing(mesh: Mesh, seed: int) -> Forcing:
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5F0C1E))
    amp = rng.uniform(-10.0, 10.0, 4)
    lo, hi = mesh.poly.min(0), mesh.poly.max(0)
    mu = []
    while len(mu) < 4:
        p = rng.uniform(lo, hi)
        if _point_in_poly(mesh.poly, p[0], p[1]):
            mu.append(p)
    sigma = rng.uniform(0.05, 0.25, 4) * mesh.R
    gq = rng.uniform(-10.0, 10.0, 6)
    return Forcing(amp, np.array(mu), sigma, gq, mesh.R)


# ----------------------------------------------------------------- problems
@dataclass
class Problem:
    """One Poisson-Dirichlet problem: mesh, eliminated system, lifted u0, parts."""
    seed: int
    mesh: Mesh
    A: CSR
    b: np.ndarray
    u0: np.ndarray
    part: np.ndarray     # int32 [N], core part of each node
    n_parts: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.mesh.n


def make_problem(seed: int, target_nodes: int, n_parts: int, jitter: float = 0.0) -> Problem:
    mesh = make_mesh(seed, target_nodes)
    fo = make_forcing(mesh, seed)
    mid = edge_midpoints(mesh)
    f_mid = fo.f(mid[..., 0], mid[..., 1])
    g = fo.g(mesh.xy[:, 0], mesh.xy[:, 1])
    A, b = assemble(mesh, f_mid, g, eliminate=True)
    u0 = np.where(mesh.dirichlet == 1, g, 0.0)
    part = partition_rcb(mesh.xy, n_parts, jitter, seed)
    return Problem(seed, mesh, A, b, u0, part, n_parts,
                   {"target_nodes": target_nodes, "jitter": jitter})


# ----------------------------------------------------------------- DSS weights
def theta_size(kbar: int, d: int) -> int:
    """Weights per model: kbar * (11 d^2 + 15 d + 1) with hidden width d (Table II)."""
    return kbar * (11 * d * d + 15 * d + 1)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """n outputs of the splitmix64 generator (Steele, Lea and Flood, 2014) from state `seed`:
    state += 0x9E3779B97F4A7C15, then the output mix of the state (two xor-shift-multiply
    rounds and a final xor-shift). Counter-based: output i depends on seed + (i + 1) * gamma only."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.arange(1, n + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def xavier_theta(seed: int, kbar: int = 30, d: int = 10) -> np.ndarray:
    """Seeded Xavier-uniform weights, zero biases (Sec. IV.B initialisation).

    Flat float32 layout, block k = 1..kbar in order, each block holding
    Phi_out {W1[d,2d+3], b1[d], W2[d,d], b2[d]}, Phi_in {same},
    Psi {W1[d,3d+1], b1[d], W2[d,d], b2[d]}, Dec {W1[d,d], b1[d], W2[1,d], b2[1]},
    matrices row-major (out, in). Matrix entries, in layout order, take consecutive
    outputs of one splitmix64 stream: u = (x >> 11) 2^-53, w = a (2u - 1) in float64
    with a = sqrt(6 / (fan_in + fan_out)), rounded to float32. The library's
    ddmgnn_model_init_xavier implements the same recipe.
    """
    shapes = []
    for _ in range(kbar):
        for _phi in range(2):
            shapes += [(d, 2 * d + 3), (d, d)]
        shapes += [(d, 3 * d + 1), (d, d), (d, d), (1, d)]
    n_mat = sum(o * i for o, i in shapes)
    u = (splitmix64(seed, n_mat) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    parts, pos = [], 0
    for fan_out, fan_in in shapes:
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(a * (2.0 * u[pos:pos + fan_out * fan_in] - 1.0))
        parts.append(np.zeros(fan_out))
        pos += fan_out * fan_in
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == theta_size(kbar, d)
    return th


# ----------------------------------------------------------------- configs
# Workload recipes. Sizes are targets: the realised node count differs by a
# few percent because the mesh is clipped to the polygon.
CONFIGS = {
    "c1": dict(target_nodes=5_000, n_parts=8, jitter=0.0, seeds=list(range(10))),
    "c2": dict(target_nodes=100_000, n_parts=150, jitter=0.15, seeds=list(range(100, 105))),
    "c3": dict(target_nodes=1_000_000, n_parts=1500, jitter=0.12, seeds=[1000, 1001, 1002]),
}
THETA_SEED = 42

# Many independent problems solved together: 64 problems with N log-uniform
# in [10k, 200k] and parts of about 600 nodes (sub-meshes of about 800 nodes
# with the overlap, all below the 2048-node kernel limit).
BATCH_CONFIGS = {
    "c4": dict(count=64, lo=10_000, hi=200_000, nodes_per_part=600, jitter=0.12, seed=2000),
}
# A stream of independent solve requests: Poisson arrivals at `rate` per
# second, N log-uniform in [lo, hi], parts of about 600 nodes.
STREAM_CONFIGS = {
    "c5": dict(count=500, rate=20.0, lo=5_000, hi=2_000_000, nodes_per_part=600, jitter=0.12, seed=3000),
}


def log_uniform_sizes(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """count integers log-uniform in [lo, hi] from a seeded generator."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), count)).astype(np.int64)


def batch_specs(name: str = "c4", count: int | None = None):
    """(seed, target_nodes, n_parts, jitter) of each problem of a batch configuration."""
    c = BATCH_CONFIGS[name]
    cnt = c["count"] if count is None else count
    sizes = log_uniform_sizes(c["seed"], c["count"], c["lo"], c["hi"])[:cnt]
    return [(c["seed"] + 1 + i, int(nn), max(1, int(round(nn / c["nodes_per_part"]))), c["jitter"])
            for i, nn in enumerate(sizes)]


def stream_specs(name: str = "c5", count: int | None = None, rate: float | None = None,
                 hi: int | None = None):
    """(arrival time in s, seed, target_nodes, n_parts, jitter) of each request of a stream."""
    c = STREAM_CONFIGS[name]
    cnt = c["count"] if count is None else count
    lam = c["rate"] if rate is None else rate
    rng = np.random.default_rng(c["seed"])
    gaps = rng.exponential(1.0 / lam, c["count"])[:cnt]
    sizes = log_uniform_sizes(c["seed"] + 1, c["count"], c["lo"], c["hi"] if hi is None else hi)[:cnt]
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[i]), c["seed"] + 2 + i, int(nn), max(1, int(round(nn / c["nodes_per_part"]))), c["jitter"])
            for i, nn in enumerate(sizes)]


def config_problem(name: str, index: int = 0) -> Problem:
    c = CONFIGS[name]
    return make_problem(c["seeds"][index], c["target_nodes"], c["n_parts"], c["jitter"])


def pack_theta(blocks: list, d: int) -> np.ndarray:
    """Flatten per-block MLP weights into the DSS weight layout (see xavier_theta).

    blocks[k] = dict(phi_out=(W1, b1, W2, b2), phi_in=(...), psi=(...), dec=(...)).
    """
    out = []
    for blk in blocks:
        for name, fan_in, fan_out in [("phi_out", 2 * d + 3, d), ("phi_in", 2 * d + 3, d),
                                      ("psi", 3 * d + 1, d), ("dec", d, 1)]:
            W1, b1, W2, b2 = blk[name]
            assert W1.shape == (d, fan_in) and b1.shape == (d,)
            assert W2.shape == (fan_out, d) and b2.shape == (fan_out,)
            out += [W1.ravel(), b1, W2.ravel(), b2]
    return np.concatenate(out).astype(np.float32)


def smoother_theta(kbar: int = 30, d: int = 10, alpha: float = 1e-3, omega=0.08,
                   out_scale: float = 1.0) -> np.ndarray:
    """Constructed (not trained) DSS weights that run damped Richardson on the graph Laplacian.

    Latent component 0 carries v. Using ReLU(x) - ReLU(-x) = x, block k realises
        phi_out_j[0] = sum_{l in N(j)} (v_l - v_j),   phi_in = 0,
        v_j <- v_j + omega_k * (c_j + phi_out_j[0]) = v_j + omega_k * (c - L v)_j,
    starting from v = 0, and the last decoder outputs out_scale * v. `omega`
    is a scalar or a length-kbar schedule. The DSS architecture and sizes are
    unchanged; only the weight values are chosen instead of drawn.
    """
    om = np.broadcast_to(np.asarray(omega, np.float64), (kbar,))
    z = lambda *s: np.zeros(s)
    blocks = []
    for k in range(kbar):
        W1 = z(d, 2 * d + 3)
        W1[0, 0], W1[0, d] = -1.0, 1.0      # unit 0: relu(v_l - v_j)
        W1[1, 0], W1[1, d] = 1.0, -1.0      # unit 1: relu(v_j - v_l)
        W2 = z(d, d)
        W2[0, 0], W2[0, 1] = 1.0, -1.0
        phi_out = (W1, z(d), W2, z(d))
        phi_in = (z(d, 2 * d + 3), z(d), z(d, d), z(d))
        P1 = z(d, 3 * d + 1)
        P1[0, d], P1[0, d + 1] = 1.0, 1.0   # relu(c + phi_out[0])
        P1[1, d], P1[1, d + 1] = -1.0, -1.0
        P2 = z(d, d)
        P2[0, 0], P2[0, 1] = om[k] / alpha, -om[k] / alpha
        psi = (P1, z(d), P2, z(d))
        D1 = z(d, d)
        D1[0, 0], D1[1, 0] = 1.0, -1.0
        D2 = z(1, d)
        D2[0, 0], D2[0, 1] = out_scale, -out_scale
        dec = (D1, z(d), D2, z(1))
        blocks.append(dict(phi_out=phi_out, phi_in=phi_in, psi=psi, dec=dec))
    return pack_theta(blocks, d)
