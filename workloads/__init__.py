"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *draws* inputs: graphs (stochastic block models and a
Gaussian-mixture k-nearest-neighbour graph), random signal blocks, start
vectors and initial centroid rows.  It contains none of the method's
arithmetic (no Laplacian, no filter, no weights kernel, no clustering): the
Gaussian-kernel weights of the kNN graph are left to each side, which receives
the squared edge lengths ``d2`` instead.

Every function is deterministic in its seed (NumPy PCG64).  Graphs are
returned as symmetric CSR with both (i, j) and (j, i) stored, column indices
strictly increasing inside each row and no self-loops, using int32 indices.

Workloads (sizes follow the synthetic settings the method is benchmarked on):
  * ``sbm``: stochastic block model with given community sizes, mean degree
    and ratio eps = p_out / p_in; node ids randomly permuted.
  * ``gmm_knn``: points from a mixture of Gaussians, symmetrised k-NN graph
    (the paper's experiments build a kNN similarity graph, Sec. 5).
  * ``signals``: R i.i.d. N(0, 1/R) columns (Sec. 3.1 and step 4 of the
    algorithm in Sec. 4.1), cast to float32 or bfloat16.
"""
from __future__ import annotations

import dataclasses
import numpy as np

BASE_SEED = 150908863


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def workload_seeds(c: int) -> dict:
    """Seeds of workload configuration c (1-based): graph, signals, k-means init, target."""
    b = BASE_SEED + 10 * c
    return {"graph": b, "signals": b + 1, "kmeans": b + 2, "target": b + 3, "lanczos": b + 4}


@dataclasses.dataclass
class Graph:
    """Symmetric CSR graph. ``w`` is None for unit weights; ``d2`` holds squared
    edge lengths for geometric graphs (weights are then a function of d2)."""
    n: int
    row_ptr: np.ndarray          # int32 [n+1]
    col_idx: np.ndarray          # int32 [nnz]
    w: np.ndarray | None = None  # float32 [nnz] or None (unit weights)
    d2: np.ndarray | None = None  # float32 [nnz] squared distances (kNN graphs)
    labels: np.ndarray | None = None  # int32 [n] ground-truth community / component
    k: int = 0

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def weights_or_ones(self) -> np.ndarray:
        if self.w is not None:
            return self.w
        return np.ones(self.nnz, dtype=np.float32)


def _csr_from_undirected(n: int, u: np.ndarray, v: np.ndarray, extra: np.ndarray | None = None):
    """Build a sorted symmetric CSR from undirected pairs (u < v or any order, no duplicates)."""
    rows = np.concatenate([u, v]).astype(np.int64)
    cols = np.concatenate([v, u]).astype(np.int64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("graph too large for int32 CSR")
    ex = None
    if extra is not None:
        ex = np.concatenate([extra, extra])[order]
    return row_ptr.astype(np.int32), cols.astype(np.int32), ex


def _sample_pairs_within(rng, n_a: int, m: int):
    """m distinct unordered pairs {x<y} of range(n_a), uniformly."""
    total = n_a * (n_a - 1) // 2
    idx = rng.choice(total, size=m, replace=False) if m > 0 else np.zeros(0, np.int64)
    idx = idx.astype(np.int64)
    # invert the row-major upper-triangle enumeration: pairs (x, y), x < y,
    # index(x, y) = x*n_a - x*(x+1)/2 + (y - x - 1)
    b = 2 * n_a - 1
    x = np.floor((b - np.sqrt(float(b) ** 2 - 8.0 * idx)) / 2.0).astype(np.int64)
    start = x * n_a - x * (x + 1) // 2
    # repair any floating-point off-by-one
    for _ in range(2):
        hi = idx < start
        x[hi] -= 1
        start = x * n_a - x * (x + 1) // 2
        nxt = (x + 1) * n_a - (x + 1) * (x + 2) // 2
        lo = idx >= nxt
        x[lo] += 1
        start = x * n_a - x * (x + 1) // 2
    y = idx - start + x + 1
    return x, y


def sbm(sizes, mean_degree: float, eps: float, seed: int, permute: bool = True) -> Graph:
    """Stochastic block model with unit weights.

    p_in = mean_degree * N / sum_a n_a((n_a - 1) + eps (N - n_a)), p_out = eps p_in.
    For every block pair the edge count is Binomial(#pairs, p) and that many
    distinct pairs are drawn without replacement.  Node ids are then permuted.
    """
    rng = rng_for(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    n = int(sizes.sum())
    denom = float(np.sum(sizes * ((sizes - 1) + eps * (n - sizes))))
    p_in = mean_degree * n / denom
    p_out = eps * p_in
    if p_in > 1.0:
        raise ValueError("mean degree too large for these community sizes")
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    us, vs = [], []
    for a in range(len(sizes)):
        na = int(sizes[a])
        if na >= 2:
            m = int(rng.binomial(na * (na - 1) // 2, p_in))
            x, y = _sample_pairs_within(rng, na, m)
            us.append(offs[a] + x)
            vs.append(offs[a] + y)
        for b in range(a + 1, len(sizes)):
            nb = int(sizes[b])
            tot = na * nb
            if tot == 0:
                continue
            m = int(rng.binomial(tot, p_out))
            idx = rng.choice(tot, size=m, replace=False).astype(np.int64) if m > 0 else np.zeros(0, np.int64)
            us.append(offs[a] + idx // nb)
            vs.append(offs[b] + idx % nb)
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    labels = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    if permute:
        perm = rng.permutation(n).astype(np.int64)  # old id -> new id
        u = perm[u]
        v = perm[v]
        new_labels = np.empty(n, dtype=np.int32)
        new_labels[perm] = labels
        labels = new_labels
    rp, ci, _ = _csr_from_undirected(n, u, v)
    return Graph(n=n, row_ptr=rp, col_idx=ci, w=np.ones(ci.shape[0], dtype=np.float32),
                 labels=labels, k=len(sizes))


def equal_sizes(n: int, k: int) -> np.ndarray:
    base = np.full(k, n // k, dtype=np.int64)
    base[: n - base.sum()] += 1
    return base


def dirichlet_sizes(n: int, k: int, alpha: float, seed: int) -> np.ndarray:
    rng = rng_for(seed)
    pi = rng.dirichlet(np.full(k, alpha))
    return rng.multinomial(n, pi).astype(np.int64)


def gmm_points(n: int, d: int, k: int, seed: int, comp_sigma: float = 1.0, mean_sigma: float = 5.0):
    """x_i = mu_{z_i} + comp_sigma * N(0, I_d), z_i uniform, mu_c ~ N(0, mean_sigma^2 I_d)."""
    rng = rng_for(seed)
    mu = rng.standard_normal((k, d)) * mean_sigma
    z = rng.integers(0, k, size=n)
    x = mu[z] + comp_sigma * rng.standard_normal((n, d))
    return x, z.astype(np.int32)


def gmm_knn(n: int, d: int, k: int, knn: int, seed: int) -> Graph:
    """Symmetrised (union) knn-nearest-neighbour graph of a Gaussian mixture.

    Stores the squared Euclidean length of every stored edge in ``d2``
    (float32); the weights are left to the caller.
    """
    from scipy.spatial import cKDTree
    x, z = gmm_points(n, d, k, seed)
    tree = cKDTree(x)
    dist, nb = tree.query(x, k=knn + 1, workers=-1)
    # drop self (distance 0 at column 0 for distinct points); keep the next knn
    src = np.repeat(np.arange(n, dtype=np.int64), knn + 1)
    dst = nb.reshape(-1).astype(np.int64)
    keep = dst != src
    src, dst = src[keep], dst[keep]
    # keep exactly knn neighbours per point (duplicates points would keep more)
    # union symmetrisation: the unordered pair set
    a = np.minimum(src, dst)
    b = np.maximum(src, dst)
    key = np.unique(a * n + b)
    u = key // n
    v = key % n
    d2 = np.sum((x[u] - x[v]) ** 2, axis=1)
    rp, ci, d2s = _csr_from_undirected(n, u, v, extra=d2)
    return Graph(n=n, row_ptr=rp, col_idx=ci, w=None, d2=d2s.astype(np.float32), labels=z, k=k)


def gmm2d_points(n: int, k: int, seed: int, min_sep: float = 5.0):
    """Planar mixture of k Gaussians with different means and spreads: means
    uniform in the square [0, 20 sqrt(k/10)]^2, each redrawn until it lies at
    least min_sep from the previous ones (visible clusters, as in the paper's
    example; at most 10000 draws per mean), sigma_c uniform in [0.3, 1.2],
    z_i uniform; x_i = mu_{z_i} + sigma_{z_i} N(0, I_2)."""
    rng = rng_for(seed)
    box = 20.0 * np.sqrt(k / 10.0)
    mu = np.zeros((k, 2))
    for c in range(k):
        for _ in range(10000):
            m = rng.uniform(0.0, box, size=2)
            if c == 0 or np.min(np.linalg.norm(mu[:c] - m, axis=1)) >= min_sep:
                break
        else:
            raise ValueError(f"cannot place {k} means {min_sep} apart in a {box:.1f} square")
        mu[c] = m
    sd = rng.uniform(0.3, 1.2, size=k)
    z = rng.integers(0, k, size=n)
    x = mu[z] + sd[z, None] * rng.standard_normal((n, 2))
    return x, z.astype(np.int32)


def knn_graph(x: np.ndarray, knn: int) -> Graph:
    """Union-symmetrised knn-nearest-neighbour pattern of the rows of x
    (self excluded), unit weights, squared edge lengths in ``d2``."""
    from scipy.spatial import cKDTree
    n = x.shape[0]
    _, nb = cKDTree(x).query(x, k=knn + 1, workers=-1)
    src = np.repeat(np.arange(n, dtype=np.int64), knn + 1)
    dst = nb.reshape(-1).astype(np.int64)
    keep = dst != src
    a = np.minimum(src[keep], dst[keep])
    b = np.maximum(src[keep], dst[keep])
    key = np.unique(a * n + b)
    u, v = key // n, key % n
    g = from_edges(n, np.stack([u, v], 1))
    # squared lengths per stored entry (row order of the CSR)
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    g.d2 = np.sum((x[rows] - x[g.col_idx]) ** 2, axis=1).astype(np.float32)
    return g


def gmm2d_knn(n: int, k: int, seed: int, knn: int | None = None) -> Graph:
    """The planar mixture's kNN graph with knn = round(ln n) by default
    (K ~ log N); ``labels`` holds the generating component."""
    x, z = gmm2d_points(n, k, seed)
    g = knn_graph(x, int(round(np.log(n))) if knn is None else knn)
    g.labels = z
    g.k = k
    return g


def unit_signals(n: int, r: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit-variance Gaussian columns drawn in float64: (float32, as float64)."""
    f32 = rng_for(seed).standard_normal((n, r)).astype(np.float32)
    return f32, f32.astype(np.float64)


def stability_pools(n: int, J: int, eta_max: int, seed: int):
    """J realisations of eta_max unit-variance columns, side by side: an
    n x (J * eta_max) float32 block (realisation j = columns j*eta_max ...)."""
    return unit_signals(n, J * eta_max, seed)


def stability_init_rows(n: int, ks, J: int, reps: int, seed: int) -> np.ndarray:
    """Initial k-means rows for every (k, realisation, replicate): int32
    [len(ks)][J][reps][max(ks)] (the first k entries are used; the rest repeat
    the first row)."""
    kmax = max(ks)
    out = np.zeros((len(ks), J, reps, kmax), dtype=np.int32)
    for q, k in enumerate(ks):
        for j in range(J):
            for t in range(reps):
                rows = init_rows(n, k, seed + 100_000 * q + 1000 * j + t)
                out[q, j, t, :k] = rows
                out[q, j, t, k:] = rows[0]
    return out


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returns the
    bfloat16 bit patterns as uint16."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    nan = np.isnan(x)
    r = r.astype(np.uint16)
    if nan.any():
        r[nan] = 0x7FC0
    return r


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)


def signals(n: int, r: int, seed: int, dtype: str = "f32"):
    """R = (r_1 | ... | r_R), entries i.i.d. N(0, 1/R) drawn in float64.

    Returns (stored, as_f64): ``stored`` is float32, or bfloat16 bit patterns
    (uint16) for dtype "bf16"; ``as_f64`` is the stored values upcast to float64
    (what an exact comparison should filter).
    """
    rng = rng_for(seed)
    r64 = rng.standard_normal((n, r)) * (1.0 / np.sqrt(r))
    f32 = r64.astype(np.float32)
    if dtype == "f32":
        return f32, f32.astype(np.float64)
    if dtype == "bf16":
        bits = bf16_round(f32)
        return bits, bf16_to_f32(bits).astype(np.float64)
    raise ValueError(dtype)


def signals_f64(n: int, r: int, seed: int) -> np.ndarray:
    """The float64 draw behind ``signals`` (before any cast)."""
    rng = rng_for(seed)
    return rng.standard_normal((n, r)) * (1.0 / np.sqrt(r))


def start_vector(n: int, seed: int) -> np.ndarray:
    """Start vector for the largest-eigenvalue iteration (float64 N(0,1))."""
    return rng_for(seed).standard_normal(n)


def init_rows(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct row indices used as the initial k-means centroids."""
    return np.sort(rng_for(seed).choice(n, size=k, replace=False)).astype(np.int32)


def unit_rows(n: int, r: int, seed: int) -> np.ndarray:
    """Rows drawn uniformly on the unit sphere of R^r (a fixed regression target), float32."""
    t = rng_for(seed).standard_normal((n, r))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return t.astype(np.float32)


# ---------------------------------------------------------------------------
# the benchmarked configurations
# ---------------------------------------------------------------------------

def workload_graph(c: int) -> Graph:
    s = workload_seeds(c)
    if c == 1:
        return sbm(equal_sizes(1000, 10), 16.0, 0.1, s["graph"])
    if c == 2:
        return sbm(equal_sizes(100_000, 20), 20.0, 0.05, s["graph"])
    if c == 3:
        return sbm(dirichlet_sizes(1_000_000, 50, 5.0, s["graph"] + 7), 30.0, 0.05, s["graph"])
    if c == 5:
        return gmm_knn(200_000, 16, 20, 10, s["graph"])
    raise ValueError(c)


WORKLOADS = {
    1: dict(name="sbm_n1e3_k10_d16_r32_p50", n=1000, k=10, r=32, p=50),
    2: dict(name="sbm_n1e5_k20_d20_r64_p100", n=100_000, k=20, r=64, p=100, steps=12, kmeans_iters=10),
    3: dict(name="sbm_n1e6_k50dir_d30_r96_p150", n=1_000_000, k=50, r=96, p=150, steps=12, kmeans_iters=10),
    4: dict(name="batch64_sbm_r48_p80_t8", r=48, p=80, trials=8, n_graphs=64),
    5: dict(name="gmm_knn10_n2e5_d16_k20_r64_p100", n=200_000, k=20, r=64, p=100, sigma=2.0, steps=12),
    # stability measure gamma(k): planar 10-Gaussian mixture, kNN with K = round(ln N),
    # k = 2..20, eta_k = 2k, J = 20 realisations
    6: dict(name="stab_gmm2d_n5000_k10_knn9_J20_k2to20_rep20", n=5000, k_true=10, ks=list(range(2, 21)), J=20,
            reps=20, p=150, steps=12, kmeans_iters=20),
    7: dict(name="stab_gmm2d_n1e5_k20_knn12_J20_k10to30_rep4", n=100_000, k_true=20, ks=list(range(10, 31)), J=20,
            reps=4, p=150, steps=12, kmeans_iters=20),
}


def stability_workload(c: int):
    """(graph, ks, etas, J, pools (float32, float64), init rows) of a stability configuration."""
    cfg = WORKLOADS[c]
    s = workload_seeds(c)
    g = gmm2d_knn(cfg["n"], cfg["k_true"], s["graph"])
    ks = cfg["ks"]
    etas = [2 * k for k in ks]
    pools = stability_pools(g.n, cfg["J"], max(etas), s["signals"])
    rows = stability_init_rows(g.n, ks, cfg["J"], cfg["reps"], s["kmeans"])
    return g, ks, etas, cfg["J"], pools, rows


def batch_specs(seed: int = BASE_SEED + 40, n_graphs: int = 64):
    """Per-graph (N, k, mean degree) of the uneven batch: N log-uniform in
    [2000, 200000], k uniform in {5..40}, mean degree uniform in [10, 30]."""
    rng = rng_for(seed)
    out = []
    for g in range(n_graphs):
        n = int(round(np.exp(rng.uniform(np.log(2000), np.log(200_000)))))
        k = int(rng.integers(5, 41))
        deg = float(rng.uniform(10, 30))
        out.append((n, k, deg))
    return out


def batch_graphs(seed: int = BASE_SEED + 40, n_graphs: int = 64, eps: float = 0.05, scale: float = 1.0):
    """The uneven batch of SBMs (equal community sizes).  ``scale`` shrinks every
    N (for CPU-sized tests)."""
    gs = []
    for g, (n, k, deg) in enumerate(batch_specs(seed, n_graphs)):
        n = max(int(n * scale), 4 * k)
        deg = min(deg, 0.5 * (n // k))
        gs.append(sbm(equal_sizes(n, k), deg, eps, seed + 1000 + g))
    return gs


# ---------------------------------------------------------------------------
# small named graphs (closed-form spectra, exact tests)
# ---------------------------------------------------------------------------

def from_edges(n: int, edges, weights=None) -> Graph:
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    extra = None if weights is None else np.asarray(weights, dtype=np.float64)
    rp, ci, ex = _csr_from_undirected(n, e[:, 0], e[:, 1], extra)
    w = np.ones(ci.shape[0], np.float32) if ex is None else ex.astype(np.float32)
    return Graph(n=n, row_ptr=rp, col_idx=ci, w=w)


def complete(n: int) -> Graph:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def cycle(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def path(n: int) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def star(n: int) -> Graph:
    return from_edges(n, [(0, i) for i in range(1, n)])


def cliques(k: int, m: int, bridges: bool = False) -> Graph:
    """k disjoint cliques of m nodes (node c*m + t in clique c); with
    ``bridges`` consecutive cliques are joined by one edge (c*m, (c+1)*m + 1)."""
    edges = [(c * m + a, c * m + b) for c in range(k) for a in range(m) for b in range(a + 1, m)]
    if bridges:
        edges += [(c * m, (c + 1) * m + 1) for c in range(k - 1)]
    g = from_edges(k * m, edges)
    g.labels = np.repeat(np.arange(k, dtype=np.int32), m)
    g.k = k
    return g


def random_weighted(n: int, p_edge: float, seed: int, isolated: int = 0) -> Graph:
    """Erdos-Renyi pattern with uniform(0.5, 2) weights; the last ``isolated``
    nodes get no edges."""
    rng = rng_for(seed)
    m = n - isolated
    iu = np.triu_indices(m, 1)
    keep = rng.random(iu[0].shape[0]) < p_edge
    u, v = iu[0][keep], iu[1][keep]
    w = rng.uniform(0.5, 2.0, size=u.shape[0])
    return from_edges(n, np.stack([u, v], 1), w)


def concat_graphs(graphs):
    """Block-diagonal concatenation: (Graph, node_off[int64 G+1]).  Columns of
    graph q are shifted by node_off[q]; weights are kept (ones if absent)."""
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    for q, g in enumerate(graphs):
        off[q + 1] = off[q] + g.n
    nnz_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    for q, g in enumerate(graphs):
        nnz_off[q + 1] = nnz_off[q] + g.nnz
    if nnz_off[-1] >= 2 ** 31:
        raise ValueError("batch too large for int32 CSR")
    rp = np.zeros(off[-1] + 1, dtype=np.int64)
    ci = np.empty(nnz_off[-1], dtype=np.int64)
    w = np.empty(nnz_off[-1], dtype=np.float32)
    for q, g in enumerate(graphs):
        rp[off[q] + 1: off[q + 1] + 1] = g.row_ptr[1:].astype(np.int64) + nnz_off[q]
        ci[nnz_off[q]: nnz_off[q + 1]] = g.col_idx.astype(np.int64) + off[q]
        w[nnz_off[q]: nnz_off[q + 1]] = g.weights_or_ones()
    big = Graph(n=int(off[-1]), row_ptr=rp.astype(np.int32), col_idx=ci.astype(np.int32), w=w)
    return big, off


def locality_order(g: Graph):
    """(permuted Graph, perm) with nodes in reverse Cuthill-McKee order
    (perm[new] = old), a bandwidth-reducing relabelling that keeps graph
    neighbours close in index space.  Data-layout preprocessing only: the
    graph is the same up to relabelling."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    A = sp.csr_matrix((np.arange(1, g.nnz + 1, dtype=np.int64), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    perm = reverse_cuthill_mckee(A, symmetric_mode=True).astype(np.int64)
    return _relabel(g, perm), perm


def block_order(g: Graph):
    """(permuted Graph, perm) with the nodes of each generating block (the
    SBM's community labels) made contiguous, blocks in label order and nodes
    in their current order inside a block (perm[new] = old).  It uses the
    generator's own labels, i.e. the best node order any partitioner could
    find for this graph; data-layout preprocessing only."""
    if g.labels is None:
        raise ValueError("block_order needs the generator's labels")
    perm = np.argsort(g.labels, kind="stable").astype(np.int64)
    return _relabel(g, perm), perm


def _relabel(g: Graph, perm: np.ndarray) -> Graph:
    import scipy.sparse as sp
    A = sp.csr_matrix((np.arange(1, g.nnz + 1, dtype=np.int64), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    B = A[perm][:, perm].tocsr()
    B.sort_indices()
    src = B.data - 1  # position of each new entry in the old arrays
    return Graph(n=g.n, row_ptr=B.indptr.astype(np.int32), col_idx=B.indices.astype(np.int32),
                 w=None if g.w is None else g.w[src], d2=None if g.d2 is None else g.d2[src],
                 labels=None if g.labels is None else g.labels[perm], k=g.k)


def seeding_draws(k: int, seed: int) -> np.ndarray:
    """k random integers uniform in [0, 2^53) (uint64): the draws of a
    k-means++ seeding, passed to both sides."""
    rng = rng_for(seed)
    return rng.integers(0, 1 << 53, size=k, dtype=np.uint64)
