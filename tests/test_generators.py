"""The seeded input generators: determinism and the shapes they promise (CPU)."""
import os
import subprocess
import sys

import numpy as np

import graphgen
import oracle


def test_rmat_deterministic_and_simple():
    a = graphgen.rmat(12, seed=1).to_csr(4, weights=True)
    b = graphgen.rmat(12, seed=1).to_csr(4, weights=True)
    c = graphgen.rmat(12, seed=2).to_csr(4)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert np.array_equal(a.weights, b.weights)
    assert not (a.num_edges == c.num_edges and np.array_equal(a.col, c.col))
    assert oracle.validate_csr(a.row_ptr, a.col, simple=True, symmetric=True) == 0


def test_thread_count_does_not_change_output():
    code = ("import graphgen, hashlib; g = graphgen.rmat(11, seed=3).to_csr(8, weights=True); "
            "print(hashlib.sha1(g.row_ptr.tobytes() + g.col.tobytes() + g.weights.tobytes()).hexdigest())")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONPATH=root)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env, text=True).strip())
    assert outs[0] == outs[1]


def test_rmat16_edge_count_and_shape():
    g = graphgen.rmat(16, seed=1).to_csr(4)
    ratio = g.num_edges / (2 * 16 * 2 ** 16)
    assert 0.84 < ratio < 0.89, ratio   # ~1.82M directed edges after dedup
    deg = g.degrees()
    assert 0.2 < np.mean(deg == 0) < 0.4
    assert deg.max() > 2000


def test_rmat_bit_marginals_unpermuted():
    """Before the id permutation an endpoint's bit is 1 with probability c+d = b+d = 0.24."""
    scale = 14
    g = graphgen.rmat(scale, seed=5, permute=False).to_csr(4)
    src = np.repeat(np.arange(g.num_vertices), np.diff(g.row_ptr).astype(np.int64))
    bits = (src[:, None] >> np.arange(scale)[None, :]) & 1
    frac = bits.mean()
    assert abs(frac - 0.24) < 0.03, frac


def test_uniform_degree_moments():
    scale, k = 14, 16
    g = graphgen.uniform(scale, (2 ** scale) * k, seed=1).to_csr(4)
    deg = g.degrees().astype(np.float64)
    assert abs(deg.mean() - 2 * k) < 0.5
    assert abs(deg.var() / deg.mean() - 1.0) < 0.1   # near-Poisson
    assert oracle.validate_csr(g.row_ptr, g.col, simple=True, symmetric=True) == 0


def test_weights_symmetric_in_range():
    g = graphgen.rmat(10, seed=1).to_csr(4, weights=True)
    assert g.weights.min() >= 1 and g.weights.max() <= 255
    assert np.array_equal(graphgen.pair_weights(g, seed=3), g.weights)
    src = np.repeat(np.arange(g.num_vertices), np.diff(g.row_ptr).astype(np.int64))
    w = {(int(u), int(v)): int(x) for u, v, x in zip(src, g.col, g.weights)}
    assert all(w[(v, u)] == x for (u, v), x in w.items())


def test_chung_lu_tail():
    n = 200000
    g = graphgen.chung_lu(n, n * 9, gamma=2.1, seed=1).to_csr(4)
    deg = g.degrees()
    d = np.sort(deg[deg > 0])[::-1]
    # log-log CCDF slope in the tail ~ -(gamma - 1)
    ranks = np.arange(1, d.shape[0] + 1)
    sel = (d >= 20) & (d <= 2000)
    slope = np.polyfit(np.log(d[sel]), np.log(ranks[sel]), 1)[0]
    assert -1.5 < slope < -0.8, slope
    assert oracle.validate_csr(g.row_ptr, g.col, simple=True, symmetric=True) == 0


def test_sources():
    g = graphgen.rmat(12, seed=1).to_csr(4)
    s = graphgen.random_sources(g, 8, seed=2)
    assert len(set(s)) == 8 and all(g.degrees()[x] > 0 for x in s)
    assert s == graphgen.random_sources(g, 8, seed=2)
    t = graphgen.degree_spread_sources(g.row_ptr, 64, seed=4)
    assert len(set(t)) == len(t) and len(t) >= 32
    degs = g.degrees()[t]
    assert degs.min() >= 1 and degs.max() == g.degrees().max()


def test_power_law_locality_order():
    h = graphgen.chung_lu(50000, 50000 * 18, gamma=2.1, seed=3, permute=False)
    before = np.sort(np.diff(h.to_csr(4).row_ptr))
    new_id = h.locality_order(run=1024, seed=3)
    g = h.to_csr(4)
    assert np.array_equal(np.sort(new_id), np.arange(50000, dtype=np.uint64))  # a bijection
    assert np.array_equal(np.sort(g.degrees()), before)                        # same degree multiset
    assert oracle.validate_csr(g.row_ptr, g.col, simple=True, symmetric=True) == 0
    # ids inside a run of 1024 keep their first-visit order: neighbours are close in id
    src = np.repeat(np.arange(g.num_vertices), g.degrees().astype(np.int64))
    near = np.mean(np.abs(src.astype(np.int64) - g.col.astype(np.int64)) < 1024)
    rnd = graphgen.chung_lu(50000, 50000 * 18, gamma=2.1, seed=3, permute=True).to_csr(4)
    src_r = np.repeat(np.arange(rnd.num_vertices), rnd.degrees().astype(np.int64))
    near_r = np.mean(np.abs(src_r.astype(np.int64) - rnd.col.astype(np.int64)) < 1024)
    assert near > 2 * near_r, (near, near_r)
    p = graphgen.power_law(40000, mean_degree=36, seed=101)
    assert 30 < p.num_edges / p.num_vertices < 42
