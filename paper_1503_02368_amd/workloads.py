"""Named benchmark workloads (seeded synthetic inputs) shared by bench.py and
the autotuner."""
from __future__ import annotations

WORKLOADS = {
    "rmat20_triangles": dict(kind="graph", pattern=3, gen="rmat", scale=20, edge_factor=16, seed=20,
                             layout=1, tau=32.0),
    "rmat18_4cliques": dict(kind="graph", pattern=4, gen="rmat", scale=18, edge_factor=16, seed=18,
                            layout=1, tau=32.0),
    "er4096_triangles": dict(kind="graph", pattern=3, gen="er", n=4096, m=32768, seed=1, layout=0,
                             tau=32.0),
    "batch_triangles": dict(kind="batch", pattern=3, graphs=20000, seed=4, layout=1, tau=32.0),
    # node-ordering study (appendix A): Chung-Lu graphs, degree exponents 1.75 .. 3
    "orderings": dict(kind="orderings", n=1 << 20, avg_degree=16.0, gammas=[1.75, 2.0, 2.5, 3.0],
                      orders=["random", "degree", "rev_degree", "bfs", "hybrid", "strong_runs"],
                      seed=30, layout=1, tau=32.0),
    # trie construction, host against GPU, on R-MAT graphs
    "build": dict(kind="build", scales=[20, 22], edge_factor=16, layout=1, tau=32.0, batch=True),
    # the unpruned relation: triangles and Lollipop on R-MAT s20 in both directions
    "unpruned": dict(kind="unpruned", scale=20, edge_factor=16, seed=20, layout=1, tau=32.0),
    # layout / algorithm ablation on R-MAT s20 (the paper's -R, -RA)
    "ablation": dict(kind="ablation", scale=20, edge_factor=16, seed=20, layout=1, tau=256.0),
    # set layouts at relation, set and block level (section 4.3): pairwise
    # intersection of sets with a dense region, then triangle counting as
    # pairwise intersections of R-MAT s20 out-sets
    "composite": dict(kind="composite", n_pairs=8192, size=4096, fracs=[0.0, 0.25, 0.5, 0.75, 1.0],
                      domain=1 << 21, density=0.5, seed=7, scale=20, edge_factor=16, graph_seed=20),
    # its composite-layout, half-dense cell alone (for profiles)
    "composite_half": dict(kind="composite", n_pairs=8192, size=4096, fracs=[0.5], domain=1 << 21,
                           density=0.5, seed=7, layouts=["composite"], levels=False),
    "served": dict(kind="served", gen="rmat", scale=22, edge_factor=16, seed=22, layout=1, tau=32.0),
}


def make_graph(w: dict):
    from paper_1503_02368_amd import inputs
    if w["gen"] == "rmat":
        return inputs.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
    return inputs.erdos_renyi_gnm(w["n"], w["m"], seed=w["seed"])


def make_batch(w: dict):
    from paper_1503_02368_amd import inputs
    return inputs.batch_chung_lu(w["graphs"], seed=w["seed"])
