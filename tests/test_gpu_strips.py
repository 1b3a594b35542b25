"""GPU strip kernels: on pixel grids the one-launch-per-phase path runs the
residual, w0 and CG-iteration phases on image strips (each workgroup walks a
strip row by row, neighbour values from an LDS ring).  The per-element
arithmetic is the row-chunk kernels', so both layouts must agree up to the
summation order of the FP64 partial sums, on every stencil width, on images
narrower than a strip and on batches; the oracle comparisons of the
one-launch-per-phase path in the other GPU test files run on strips too."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, gpu_graph, oracle_graph, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


# (name, H, W, stencil, d): every stencil width, ragged sizes, images narrower
# than one strip, tall and flat images, and d = 32 (strips of 12 or 14 pixels)
CASES = [
    ("voronoi96x80_8nbr", None, None, None, None),
    ("voronoi48x40_r2", None, None, None, None),
    ("voronoi64_4nbr", None, None, None, None),
    ("ragged37x41_8", 37, 41, 8, 6),
    ("narrow300x7_r2", 300, 7, -2, 5),
    ("flat5x333_4", 5, 333, 4, 3),
    ("wide33x70_d32_r2", 33, 70, -2, 32),
    ("multi23x95_8_d16", 23, 95, 8, 16),
]


def case_workload(case):
    name, H, W, st, d = case
    if H is None:
        return synth.make_workload(name, 0)
    return synth.grid_workload(name, H, W, 4, 0.05, 11, gradient=0.2, stencil=st, d=d, n_inner=3, n_outer=2)


def run(wl, monkeypatch, strips, fp64, n_outer=2, lam=30.0, r=3.0, graphs=False, tol=None):
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_STRIPS", "1" if strips else "0")
    G = gpu_graph(wl)
    if tol is None:
        tol = 1e-10 if fp64 else 1e-6
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=3, tol=tol, maxit=3000, fp64=fp64,
               persistent=False, graphs=graphs)
    info = S.solve(n_outer, info=True)
    return info, {k: to_np(S.get(k)) for k in ("Y", "P", "B")}


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_strips_match_row_chunks(case, fp64, monkeypatch):
    wl = case_workload(case)
    banner(f"strips vs row chunks {case[0]} fp64={fp64}")
    i1, on = run(wl, monkeypatch, True, fp64)
    i0, off = run(wl, monkeypatch, False, fp64)
    assert i1["flags"] & 2, "the strip kernels did not run"
    assert not (i0["flags"] & 2)
    worst = max(rel(on[k], off[k]) for k in ("Y", "P"))
    eB = np.linalg.norm(on["B"] - off["B"]) / np.linalg.norm(off["P"])
    bound = 1e-10 if fp64 else 1e-5
    print(f"Y/P rel {worst:.2e}, B {eB:.2e}; CG iterations {i1['cg_iters_total']} vs {i0['cg_iters_total']}")
    assert worst <= bound and eB <= bound
    if fp64:
        assert i1["cg_iters_total"] == i0["cg_iters_total"]
    else:
        assert abs(i1["cg_iters_total"] - i0["cg_iters_total"]) <= max(2, i0["cg_iters_total"] // 50)


def test_strips_outer_step_matches_oracle(monkeypatch):
    """Two SOC iterations on strips in FP64 (ragged 8-neighbour image) against the oracle."""
    wl = case_workload(CASES[3])
    banner("strips vs oracle (ragged 37x41)")
    g = oracle_graph(wl)
    lam, r = 30.0, 3.0
    ref = O.pfe_run(g, wl.y0, lam, r, 2, 3)
    info, got = run(wl, monkeypatch, True, True, lam=lam, r=r, tol=1e-12)
    assert info["flags"] & 2
    e = rel(got["P"], ref.P)
    print(f"P rel err vs oracle {e:.2e}")
    assert e <= 1e-8


def test_strips_graph_replay_bitwise(monkeypatch):
    """PCG iterations on strips replayed from HIP graphs give bitwise the
    host-launched iteration."""
    wl = synth.make_workload("voronoi96x80_8nbr", 0)
    banner("strips + graph replay")
    out = [run(wl, monkeypatch, True, False, graphs=g) for g in (True, False)]
    assert out[0][0]["cg_iters_total"] == out[1][0]["cg_iters_total"]
    for k in ("Y", "P", "B"):
        assert np.array_equal(out[0][1][k], out[1][1][k])


def test_strips_deterministic(monkeypatch):
    wl = synth.make_workload("voronoi48x40_r2", 0)
    banner("strips determinism")
    a = run(wl, monkeypatch, True, False)[1]
    b = run(wl, monkeypatch, True, False)[1]
    for k in ("Y", "P", "B"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("fp64", [True, False])
def test_strips_batch_matches_solo(fp64, monkeypatch):
    """A batch of uneven images on strips == each image alone on strips."""
    from paper_1612_06496_amd import Graph, Solver
    monkeypatch.setenv("PFE_STRIPS", "1")
    wls = synth.make_batch("voronoi_batch5_8nbr")
    banner(f"strips batch == solo fp64={fp64}")
    parts = [gpu_graph(w) for w in wls]
    U = Graph.union(parts)
    kw = dict(lam=20.0, r=2.0, n_inner=wls[0].n_inner, tol=1e-11 if fp64 else 1e-6, maxit=3000, fp64=fp64,
              persistent=False)
    S = Solver(U, np.concatenate([w.y0 for w in wls]), **kw)
    info = S.solve(2, info=True)
    assert info["flags"] & 2
    got = {k: to_np(S.get(k)) for k in ("Y", "P")}
    row0, _ = U.segments
    worst = 0.0
    for k, (w, p) in enumerate(zip(wls, parts)):
        Ss = Solver(p, w.y0, **kw)
        Ss.solve(2)
        sl = slice(row0[k], row0[k + 1])
        worst = max(worst, rel(got["Y"][sl], to_np(Ss.get("Y"))), rel(got["P"][sl], to_np(Ss.get("P"))))
    bound = 1e-8 if fp64 else 1e-5
    print(f"worst segment rel err {worst:.2e} (bound {bound})")
    assert worst <= bound


def test_pcg_on_strips_matches_direct_solve(monkeypatch):
    """The standalone PCG call on strips (FP64, 5x5 window) reaches the direct
    solution within the condition-number bound of its stopping rule."""
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_STRIPS", "1")
    wl = synth.make_workload("voronoi48x40_r2", 0)
    banner("pfe_pcg on strips vs direct solve")
    g = oracle_graph(wl)
    lam, r, tol = 40.0, 2.0, 1e-12
    S = Solver(gpu_graph(wl), wl.y0, lam=lam, r=r, n_inner=2, tol=tol, maxit=5000, fp64=True, persistent=False)
    A = O.system_matrix(g, lam, r)
    rhs = np.random.default_rng(5).normal(size=(g.n, wl.d))
    x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
    exact = O.DirectSolver(A)(rhs)
    kappa = O.jacobi_condition_number(A)
    e = rel(to_np(x), exact)
    print(f"rel err {e:.2e}, kappa {kappa:.1f}, iterations {iters.max()}")
    assert info["rel_res_max"] <= tol
    assert e <= kappa * tol * 4
    _, it_o, _ = O.pcg(A, rhs, np.zeros_like(rhs), 1.0 / A.diagonal(), tol, 5000)
    assert np.all(np.abs(iters - it_o) <= 1)


def test_autotune_offers_strips(monkeypatch):
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_STRIPS", "1")
    wl = synth.make_workload("voronoi96x80_8nbr", 0)
    banner("autotune with strips")
    S = Solver(gpu_graph(wl), wl.y0, lam=30.0, r=3.0, n_inner=3, tol=1e-6, maxit=1000)
    res = S.autotune(1)
    assert any(r["strips"] == 1 and r["persistent"] == 0 for r in res), res
    assert sum(r["chosen"] for r in res) == 1


@pytest.mark.parametrize("stencil,d", [(8, 4), (-2, 5), (4, 3)])
def test_learned_pcg_strips_match_row_chunks(stencil, d, monkeypatch):
    """PCG with a (non-identity) learned factor: the three strip phases per
    iteration give the row-chunk phases' iterate and iteration counts."""
    from paper_1612_06496_amd import Mpnn, Solver
    banner(f"learned PCG strips vs row chunks stencil={stencil}")
    wl = synth.grid_workload("t", 45, 101, 6, 0.05, 3, stencil=stencil, d=d)
    th = np.random.default_rng(1).normal(0.0, 0.3, size=Mpnn.NPARAMS)
    th[Mpnn.NPARAMS - 1] = np.log(np.e - 1.0)
    rhs = np.random.default_rng(2).normal(size=(wl.n, d))
    out = []
    for strips in ("1", "0"):
        monkeypatch.setenv("PFE_STRIPS", strips)
        S = Solver(gpu_graph(wl), wl.y0, lam=20.0, r=1.0, n_inner=2, tol=1e-10, maxit=5000, fp64=True,
                   persistent=False)
        S.set_learned(Mpnn(th.astype(np.float32)))
        x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
        out.append((to_np(x), np.asarray(iters), info))
    e = rel(out[0][0], out[1][0])
    print(f"rel diff {e:.2e}; iterations {out[0][1].tolist()} vs {out[1][1].tolist()}")
    assert np.all(np.abs(out[0][1] - out[1][1]) <= 1)
    assert e <= 1e-9
    assert out[0][2]["rel_res_max"] <= 1e-10


@pytest.mark.parametrize("stencil,d,fp64", [(8, 4, True), (-2, 5, True), (4, 3, True), (-2, 16, False), (8, 10, False)])
def test_one_pass_factor_pcg_matches_two_pass(stencil, d, fp64):
    """Factor-preconditioned PCG on image strips: the one-pass
    Chronopoulos-Gear iteration (u = M^{-1} r and w = A u formed through three
    LDS rings) against the two-pass iteration (A p, then the factor apply with
    the x, r update): the same solution to the tolerance and the same
    iteration counts within one, on ragged images."""
    from paper_1612_06496_amd import Mpnn, Solver
    banner(f"one-pass vs two-pass factor PCG stencil={stencil} d={d} fp64={fp64}")
    wl = synth.grid_workload("t", 45, 101, 6, 0.05, 3, stencil=stencil, d=d)
    th = np.random.default_rng(1).normal(0.0, 0.3, size=Mpnn.NPARAMS)
    th[Mpnn.NPARAMS - 1] = np.log(np.e - 1.0)
    rhs = np.random.default_rng(2).normal(size=(wl.n, d))
    tol = 1e-10 if fp64 else 1e-6
    out = []
    for one_pass in (True, False):
        S = Solver(gpu_graph(wl), wl.y0, lam=20.0, r=1.0, n_inner=2, tol=tol, maxit=5000, fp64=fp64,
                   persistent=False, graphs=one_pass)
        S.set_launch_shape(persistent=False, strips=1, one_pass=one_pass)
        S.set_learned(Mpnn(th.astype(np.float32)))
        x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
        out.append((to_np(x), np.asarray(iters), info))
        S.close()
    e = rel(out[0][0], out[1][0])
    print(f"rel diff {e:.2e}; iterations {out[0][1].tolist()} vs {out[1][1].tolist()}; "
          f"rel res {out[0][2]['rel_res_max']:.2e}")
    assert np.all(np.abs(out[0][1] - out[1][1]) <= 1)
    assert out[0][2]["rel_res_max"] <= tol
    assert e <= (1e-8 if fp64 else 1e-4)


def run_eu(wl_or_graph, y0, monkeypatch, eu_px, fp64, keep_split, inner_steps):
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_EU_PX", "1" if eu_px else "0")
    # the edge update alone (not fused with the next residual, which has its own test)
    monkeypatch.setenv("PFE_EUR_PX", "0")
    monkeypatch.setenv("PFE_STRIPS", "1")
    S = Solver(wl_or_graph, y0, lam=30.0, r=3.0, n_inner=3, tol=1e-10 if fp64 else 1e-6, maxit=3000, fp64=fp64,
               persistent=False, keep_split=keep_split)
    S.solve(1)
    for _ in range(inner_steps):
        S.step("inner")
    out = {k: S.get(k).cpu().numpy() for k in ("Y", "P", "B", "b") + (("d",) if keep_split else ())}
    S.close()
    return out


EU_CASES = ["voronoi96x80_8nbr", "voronoi48x40_r2", "voronoi64_4nbr", "narrow300x7_r2", "wide33x70_d32_r2",
            "multi23x95_8_d16"]


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("name", EU_CASES + ["batch5", "edges_d4", "edges_d5"])
def test_pixel_edge_update_bitwise_equals_phase_kernels(name, fp64, monkeypatch):
    """The per-pixel edge update (one thread per pixel and 1, 2 or 4 columns;
    neighbours from the stencil offsets on one image, from the slot columns on a
    batch and on edge-list graphs, whose b and d are stored per slot) does the
    phase kernels' arithmetic element by element in the same slot order: Y, P,
    B, b and d after a SOC iteration and two inner steps (both b-buffer
    parities) are bitwise those of the strip / row-chunk edge update."""
    from paper_1612_06496_amd import Graph
    banner(f"per-pixel edge update == phase kernels: {name} fp64={fp64}")
    if name == "batch5":
        wls = synth.make_batch("voronoi_batch5_8nbr")
        G = Graph.union([gpu_graph(w) for w in wls])
        y0 = np.concatenate([w.y0 for w in wls])
    elif name.startswith("edges"):
        # an edge-list graph: b and d per slot, the slot columns of the general layout
        wl = synth.edges_workload("gmm_small", 5000, 8, 4, 6, 3, d=int(name[-1]), n_outer=2, n_inner=3)
        G, y0 = gpu_graph(wl), wl.y0
    else:
        wl = case_workload(next(c for c in CASES if c[0] == name))
        G, y0 = gpu_graph(wl), wl.y0
    keep = name in ("voronoi48x40_r2", "batch5", "edges_d4")
    a = run_eu(G, y0, monkeypatch, True, fp64, keep, 2)
    b = run_eu(G, y0, monkeypatch, False, fp64, keep, 2)
    for k in a:
        assert np.array_equal(a[k], b[k]), f"{k} differs: max {np.abs(a[k] - b[k]).max():.3e}"
    print("bitwise equal:", sorted(a))
