"""GPU pixel launches: on a one-image pixel grid the Jacobi PCG phases can run
as per-pixel kernels (one thread per pixel and 1, 2 or 4 columns, neighbours
through L2): the residual, w0 = A u0, and each CG iteration in two passes (the
own-row updates storing u' = r'/diag(A), then w' = A u').  The per-element
arithmetic is the row-chunk phases', so the results agree with the strip and
row-chunk launches up to the summation order of the FP64 partial sums, and with
the oracle (Eq. 13 solved by Jacobi-PCG, Algorithms 1-2)."""
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


# every stencil width, ragged sizes, d with 1, 2 and 4 columns per thread
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


def run(wl, monkeypatch, pixel, fp64, strips=1, n_outer=2, lam=30.0, r=3.0, graphs=False, tol=None):
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_PIXEL", "1" if pixel else "0")
    monkeypatch.setenv("PFE_STRIPS", str(strips))
    G = gpu_graph(wl)
    if tol is None:
        tol = 1e-10 if fp64 else 1e-6
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=3, tol=tol, maxit=3000, fp64=fp64, persistent=False, graphs=graphs)
    info = S.solve(n_outer, info=True)
    out = {k: to_np(S.get(k)) for k in ("Y", "P", "B")}
    S.close()
    G.close()
    return info, out


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pixel_launch_matches_strips_and_row_chunks(case, fp64, monkeypatch):
    wl = case_workload(case)
    banner(f"pixel launch vs strips / row chunks {case[0]} fp64={fp64}")
    ip, px = run(wl, monkeypatch, True, fp64)
    assert ip["flags"] & 4, "the pixel kernels did not run"
    assert ip["flags"] & 8, "the edge updates did not form the next residual"
    bound = 1e-10 if fp64 else 1e-5
    for strips in (1, 0):
        io, other = run(wl, monkeypatch, False, fp64, strips=strips)
        assert not (io["flags"] & 4)
        worst = max(rel(px[k], other[k]) for k in ("Y", "P"))
        eB = np.linalg.norm(px["B"] - other["B"]) / np.linalg.norm(other["P"])
        print(f"strips={strips}: Y/P rel {worst:.2e}, B {eB:.2e}; CG iterations "
              f"{ip['cg_iters_total']} vs {io['cg_iters_total']}")
        assert worst <= bound and eB <= bound
        if fp64:
            assert ip["cg_iters_total"] == io["cg_iters_total"]
        else:
            assert abs(ip["cg_iters_total"] - io["cg_iters_total"]) <= max(2, io["cg_iters_total"] // 50)


def test_pixel_launch_outer_step_matches_oracle(monkeypatch):
    """Two SOC iterations by pixel launches in FP64 (ragged 8-neighbour image) against the oracle."""
    wl = case_workload(CASES[3])
    banner("pixel launch vs oracle (ragged 37x41)")
    g = oracle_graph(wl)
    lam, r = 30.0, 3.0
    ref = O.pfe_run(g, wl.y0, lam, r, 2, 3)
    info, got = run(wl, monkeypatch, True, True, lam=lam, r=r, tol=1e-12)
    assert info["flags"] & 4
    e = rel(got["P"], ref.P)
    print(f"P rel err vs oracle {e:.2e}")
    assert e <= 1e-8


@pytest.mark.parametrize("precond", ["jacobi", "fsai"])
@pytest.mark.parametrize("pixel", [1, 0])
@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("name", ["voronoi48x40_r2", "voronoi96x80_8nbr", "voronoi64_4nbr", "ragged37x41_8"])
def test_fused_edge_update_residual_matches_separate_kernels(name, fp64, pixel, precond, monkeypatch):
    """An SOC iteration run in one call (each edge update but the last also
    forms the next solve's residual r0 = rhs - A Y, u0 = r0 / diag(A) and the
    CG start: k_eur_px) against the same iteration one inner step per call (edge
    update, then the residual kernel of the next solve), with the PCG in per-row
    launches (pixel = 1) or on strips (the fused kernel on the per-row
    partition): per-row bitwise equal in FP64, where the fused kernel sums the
    slots in the residual kernel's order; strips in FP64 within 1e-12 (the
    residual norms are summed over other workgroups) and CG iterations within
    1; in FP32 (slots visited in pairs) Y, P within 1e-5 (B relative to P) and
    CG iterations within 2.  Jacobi PCG, and the FSAI factor (whose fused edge
    updates also store the right-hand side for the Jacobi fallback)."""
    from paper_1612_06496_amd import Solver
    wl = case_workload(next(c for c in CASES if c[0] == name))
    banner(f"fused edge update + residual vs separate kernels: {name} fp64={fp64} pixel={pixel} {precond}")
    monkeypatch.setenv("PFE_PIXEL", str(pixel))
    monkeypatch.setenv("PFE_STRIPS", "1")
    G = gpu_graph(wl)
    res = []
    for fused in (True, False):
        S = Solver(G, wl.y0, lam=30.0, r=3.0, n_inner=4, tol=1e-10 if fp64 else 1e-6, maxit=3000, fp64=fp64,
                   persistent=False)
        if precond == "fsai":
            S.set_fsai()
        S.solve(1)                     # a first SOC iteration, so that P, B and b are not trivial
        if fused:
            info = S.solve(1, info=True)
        else:
            iters = 0
            for _ in range(4):
                step = S.step("inner", info=True)
                assert not step["flags"] & 8
                iters += step["cg_iters_total"]
            info = S.step("outer", info=True)
            info["cg_iters_total"] += iters
            assert not info["flags"] & 8
        res.append((info, {k: to_np(S.get(k)) for k in ("Y", "P", "B")}))
        S.close()
    G.close()
    (i1, o1), (i2, o2) = res
    assert i1["flags"] & 8 and i1["flags"] & (4 if pixel else 2)
    print("CG iterations fused / separate:", i1["cg_iters_total"], i2["cg_iters_total"])
    if fp64 and not pixel:
        assert abs(i1["cg_iters_total"] - i2["cg_iters_total"]) <= 1
        for k in ("Y", "P"):
            assert rel(o1[k], o2[k]) <= 1e-12, k
    elif fp64:
        assert i1["cg_iters_total"] == i2["cg_iters_total"]
        for k in o1:
            assert np.array_equal(o1[k], o2[k]), k
    else:
        assert abs(i1["cg_iters_total"] - i2["cg_iters_total"]) <= 2
        for k in ("Y", "P"):
            assert rel(o1[k], o2[k]) <= 1e-5, k
        # B = Z - P is a small difference of O(1) quantities: relative to P
        assert np.linalg.norm(o1["B"] - o2["B"]) / np.linalg.norm(o2["P"]) <= 1e-5


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("d,n", [(4, 5000), (5, 5000), (4, 900)])
def test_fused_edge_update_residual_general_graph_bitwise(d, n, fp64, monkeypatch):
    """Per-row launches on an edge-list graph (general slot layout, b per slot):
    an SOC iteration in one call (each edge update but the last also forms the
    next residual, summing w^2 y_j in the residual kernel's slot order) equals,
    bitwise in FP32 and FP64, the same iteration one inner step per call."""
    from paper_1612_06496_amd import Solver
    wl = edge_workload(d, n)
    banner(f"fused edge update + residual, edge-list graph d={d} n={n} fp64={fp64}")
    monkeypatch.setenv("PFE_PIXEL", "1")
    G = gpu_graph(wl)
    res = []
    for fused in (True, False):
        S = Solver(G, wl.y0, lam=30.0, r=3.0, n_inner=3, tol=1e-10 if fp64 else 1e-6, maxit=3000, fp64=fp64,
                   persistent=False)
        S.solve(1)
        if fused:
            info = S.solve(1, info=True)
        else:
            iters = sum(S.step("inner", info=True)["cg_iters_total"] for _ in range(3))
            info = S.step("outer", info=True)
            info["cg_iters_total"] += iters
        res.append((info, {k: to_np(S.get(k)) for k in ("Y", "P", "B")}))
        S.close()
    G.close()
    (i1, o1), (i2, o2) = res
    assert i1["flags"] & 4 and i1["flags"] & 8 and not i2["flags"] & 8
    assert i1["cg_iters_total"] == i2["cg_iters_total"]
    for k in o1:
        assert np.array_equal(o1[k], o2[k]), k


def test_pixel_launch_graph_replay_bitwise_and_deterministic(monkeypatch):
    """CG iterations replayed from HIP graphs (two nodes per iteration) give
    bitwise the host-launched ones, and a rerun gives bitwise the same state."""
    wl = synth.make_workload("voronoi48x40_r2", 0)
    banner("pixel launch + graph replay, determinism")
    out = [run(wl, monkeypatch, True, False, graphs=g) for g in (True, False, False)]
    assert out[0][0]["cg_iters_total"] == out[1][0]["cg_iters_total"]
    for k in ("Y", "P", "B"):
        assert np.array_equal(out[0][1][k], out[1][1][k])
        assert np.array_equal(out[1][1][k], out[2][1][k])


@pytest.mark.parametrize("name,d", [("voronoi48x40_r2", None), ("voronoi64_4nbr", None), ("voronoi64_4nbr", 3)])
def test_pixel_launch_pcg_matches_direct_solve(name, d, monkeypatch):
    """The standalone PCG call by pixel launches (FP64) reaches the direct
    solution within the condition-number bound of its stopping rule, in the
    oracle's Jacobi-PCG iteration count (+-1)."""
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_PIXEL", "1")
    wl = synth.make_workload(name, 0)
    y0 = wl.y0 if d is None else wl.y0[:, :d]
    banner(f"pfe_pcg by pixel launches vs direct solve: {name}")
    g = oracle_graph(wl)
    lam, r, tol = 40.0, 2.0, 1e-12
    G = gpu_graph(wl)
    S = Solver(G, y0, lam=lam, r=r, n_inner=2, tol=tol, maxit=5000, fp64=True, persistent=False)
    A = O.system_matrix(g, lam, r)
    rhs = np.random.default_rng(5).normal(size=(g.n, y0.shape[1]))
    x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
    assert info["flags"] & 4
    exact = O.DirectSolver(A)(rhs)
    kappa = O.jacobi_condition_number(A)
    e = rel(to_np(x), exact)
    print(f"rel err {e:.2e}, kappa {kappa:.1f}, iterations {iters.max()}")
    assert info["rel_res_max"] <= tol
    assert e <= kappa * tol * 4
    _, it_o, _ = O.pcg(A, rhs, np.zeros_like(rhs), 1.0 / A.diagonal(), tol, 5000)
    assert np.all(np.abs(iters - it_o) <= 1)
    S.close()
    G.close()


def test_autotune_offers_pixel_launches(monkeypatch):
    from paper_1612_06496_amd import Solver
    monkeypatch.delenv("PFE_PIXEL", raising=False)
    wl = synth.make_workload("voronoi96x80_8nbr", 0)
    banner("autotune with pixel launches")
    G = gpu_graph(wl)
    S = Solver(G, wl.y0, lam=30.0, r=3.0, n_inner=3, tol=1e-6, maxit=1000)
    res = S.autotune(1)
    assert any(r["pixel"] == 1 and r["persistent"] == 0 for r in res), res
    assert sum(r["chosen"] for r in res) == 1
    S.set_launch_shape(persistent=False, pixel=True)
    info = S.solve(1, info=True)
    assert info["flags"] & 4
    S.close()
    G.close()


@pytest.mark.parametrize("fp64", [True, False])
def test_pixel_launch_batch_matches_solo_and_strips(fp64, monkeypatch):
    """A batch of uneven images by pixel launches (each workgroup a row range of
    one image, its geometry and its segment's CG scalars): every image equals
    its solo pixel-launch run, and the batch equals the strip launches."""
    from paper_1612_06496_amd import Graph, Solver
    wls = synth.make_batch("voronoi_batch5_8nbr")
    banner(f"pixel-launch batch == solo and == strips, fp64={fp64}")
    kw = dict(lam=20.0, r=2.0, n_inner=wls[0].n_inner, tol=1e-11 if fp64 else 1e-6, maxit=3000, fp64=fp64,
              persistent=False)
    y0 = np.concatenate([w.y0 for w in wls])
    out = {}
    for pixel in (1, 0):
        monkeypatch.setenv("PFE_PIXEL", str(pixel))
        monkeypatch.setenv("PFE_STRIPS", "1")
        parts = [gpu_graph(w) for w in wls]
        U = Graph.union(parts)
        S = Solver(U, y0, **kw)
        info = S.solve(2, info=True)
        assert bool(info["flags"] & 4) == bool(pixel) and bool(info["flags"] & 2) != bool(pixel)
        out[pixel] = {k: to_np(S.get(k)) for k in ("Y", "P")}
        row0, _ = U.segments
        if pixel:
            worst = 0.0
            for k, (w, p) in enumerate(zip(wls, parts)):
                Ss = Solver(p, w.y0, **kw)
                Ss.solve(2)
                sl = slice(row0[k], row0[k + 1])
                worst = max(worst, rel(out[1]["Y"][sl], to_np(Ss.get("Y"))), rel(out[1]["P"][sl], to_np(Ss.get("P"))))
                Ss.close()
        S.close()
    bound = 1e-8 if fp64 else 1e-5
    vs_strips = max(rel(out[1][k], out[0][k]) for k in ("Y", "P"))
    print(f"worst segment vs solo {worst:.2e}; batch vs strips {vs_strips:.2e} (bound {bound})")
    assert worst <= bound and vs_strips <= bound


def test_pixel_launch_shape_checks_and_factor_preconditioners(monkeypatch):
    """set_launch_shape rejects two workgroups per CU on a graph too small for
    them and sizes other than 1 and 2; a factor-preconditioned (FSAI) solve on a
    pixel grid runs by pixel launches too, and on an edge-list graph it keeps
    the row chunks."""
    from paper_1612_06496_amd import Solver
    from paper_1612_06496_amd import _lib as L
    monkeypatch.setenv("PFE_PIXEL", "1")
    banner("pixel launches: shape checks, factor preconditioners")
    wl = synth.make_workload("voronoi48x40_r2", 0)
    G = gpu_graph(wl)
    S = Solver(G, wl.y0, lam=20.0, r=2.0, n_inner=2, tol=1e-6, persistent=False)
    with pytest.raises(L.PFEError):
        S.set_launch_shape(persistent=False, pixel=2)    # too few rows for more workgroups than CUs
    with pytest.raises(L.PFEError):
        S.set_launch_shape(persistent=False, pixel=3)
    S.set_fsai()
    info = S.solve(1, info=True)
    assert info["flags"] & 4
    S.close()
    G.close()
    from paper_1612_06496_amd import Mpnn
    wle = edge_workload(4)
    G = gpu_graph(wle)
    S = Solver(G, wle.y0, lam=20.0, r=2.0, n_inner=2, tol=1e-6, persistent=False)
    net = Mpnn(None)
    S.set_learned(net)
    info = S.solve(1, info=True)
    assert not (info["flags"] & 4)
    S.close()
    net.close()
    G.close()


def edge_workload(d, n=5000):
    # 5000 points: several 512-thread workgroups of rows even at four columns per thread
    return synth.edges_workload("gmm_small", n, 8, 4, 6, 3, d=d, n_outer=2, n_inner=3)


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("d,n", [(4, 5000), (5, 5000), (4, 900)])
def test_row_launch_general_graph_matches_row_chunks(d, n, fp64, monkeypatch):
    """Per-row launches on an edge-list graph (k-NN, general slot layout; the
    neighbours from the slot columns): two SOC iterations equal the row-chunk
    launches' up to the FP64 summation order (900 points: fewer workgroups
    than XCDs)."""
    wl = edge_workload(d, n)
    banner(f"row launch vs row chunks, edge-list graph d={d} fp64={fp64}")
    ip, px = run(wl, monkeypatch, True, fp64, strips=0)
    assert ip["flags"] & 4, "the per-row kernels did not run"
    io, rc = run(wl, monkeypatch, False, fp64, strips=0)
    assert not (io["flags"] & 4)
    bound = 1e-10 if fp64 else 1e-5
    worst = max(rel(px[k], rc[k]) for k in ("Y", "P"))
    eB = np.linalg.norm(px["B"] - rc["B"]) / np.linalg.norm(rc["P"])
    print(f"Y/P rel {worst:.2e}, B {eB:.2e}; CG iterations {ip['cg_iters_total']} vs {io['cg_iters_total']}")
    assert worst <= bound and eB <= bound
    if fp64:
        assert ip["cg_iters_total"] == io["cg_iters_total"]
    else:
        assert abs(ip["cg_iters_total"] - io["cg_iters_total"]) <= max(2, io["cg_iters_total"] // 50)


def test_row_launch_general_graph_pcg_matches_direct_solve(monkeypatch):
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_PIXEL", "1")
    wl = edge_workload(4)
    banner("pfe_pcg by per-row launches on an edge-list graph vs direct solve")
    g = oracle_graph(wl)
    lam, r, tol = 40.0, 2.0, 1e-12
    G = gpu_graph(wl)
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=2, tol=tol, maxit=5000, fp64=True, persistent=False)
    A = O.system_matrix(g, lam, r)
    rhs = np.random.default_rng(7).normal(size=(g.n, wl.y0.shape[1]))
    x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
    assert info["flags"] & 4
    exact = O.DirectSolver(A)(rhs)
    kappa = O.jacobi_condition_number(A)
    e = rel(to_np(x), exact)
    print(f"rel err {e:.2e}, kappa {kappa:.1f}, iterations {iters.max()}")
    assert info["rel_res_max"] <= tol
    assert e <= kappa * tol * 4
    _, it_o, _ = O.pcg(A, rhs, np.zeros_like(rhs), 1.0 / A.diagonal(), tol, 5000)
    assert np.all(np.abs(iters - it_o) <= 1)
    S.close()
    G.close()


FACTOR_CASES = [(8, 4, True, "learned"), (-2, 5, True, "learned"), (4, 3, True, "fsai"), (-2, 16, True, "fsai"),
                (-2, 16, False, "learned"), (8, 10, False, "fsai")]


@pytest.mark.parametrize("stencil,d,fp64,pre", FACTOR_CASES)
def test_pixel_factor_pcg_matches_strips(stencil, d, fp64, pre, monkeypatch):
    """Factor-preconditioned PCG (learned G or FSAI) by pixel launches, three
    per-pixel passes per iteration (p and q = A p; x, r' and y1 = Gt D_A^{-1/2} r';
    z = D_A^{-1/2} Gt^T y1), against the strip launches on every stencil width
    and with 1, 2 and 4 columns per thread: the iterate and the iteration
    counts of the standalone PCG call."""
    from paper_1612_06496_amd import Mpnn, Solver
    banner(f"{pre} PCG by pixel launches vs strips: stencil={stencil} d={d} fp64={fp64}")
    wl = synth.grid_workload("t", 45, 101, 6, 0.05, 3, stencil=stencil, d=d)
    th = np.random.default_rng(1).normal(0.0, 0.3, size=Mpnn.NPARAMS)
    th[Mpnn.NPARAMS - 1] = np.log(np.e - 1.0)
    rhs = np.random.default_rng(2).normal(size=(wl.n, d))
    tol = 1e-10 if fp64 else 1e-6
    out = []
    for pixel in ("1", "0"):
        monkeypatch.setenv("PFE_PIXEL", pixel)
        monkeypatch.setenv("PFE_STRIPS", "1")
        G = gpu_graph(wl)
        S = Solver(G, wl.y0, lam=20.0, r=1.0, n_inner=2, tol=tol, maxit=5000, fp64=fp64, persistent=False)
        net = None
        if pre == "learned":
            net = Mpnn(th.astype(np.float32))
            S.set_learned(net)
        else:
            S.set_fsai()
        x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
        assert bool(info["flags"] & 4) == (pixel == "1")
        assert info["fallbacks"] == 0
        out.append((to_np(x), np.asarray(iters), info))
        S.close()
        if net is not None:
            net.close()
        G.close()
    e = rel(out[0][0], out[1][0])
    print(f"rel diff {e:.2e}; iterations {out[0][1].tolist()} vs {out[1][1].tolist()}")
    assert np.all(np.abs(out[0][1] - out[1][1]) <= (1 if fp64 else 2))
    assert e <= (1e-9 if fp64 else 1e-4)
    assert out[0][2]["rel_res_max"] <= tol


def test_pixel_factor_pcg_graph_replay_bitwise_and_direct_solve(monkeypatch):
    """FSAI PCG by pixel launches: replayed from HIP graphs (three nodes per
    iteration) bitwise equal to host launches, and the solution of the direct
    solve within the condition-number bound of the stopping rule."""
    from paper_1612_06496_amd import Solver
    monkeypatch.setenv("PFE_PIXEL", "1")
    wl = synth.make_workload("voronoi48x40_r2", 0)
    banner("FSAI PCG by pixel launches: graph replay, direct solve")
    g = oracle_graph(wl)
    lam, r, tol = 40.0, 2.0, 1e-12
    rhs = np.random.default_rng(5).normal(size=(g.n, wl.y0.shape[1]))
    res = []
    for graphs in (True, False):
        G = gpu_graph(wl)
        S = Solver(G, wl.y0, lam=lam, r=r, n_inner=2, tol=tol, maxit=5000, fp64=True, persistent=False,
                   graphs=graphs)
        S.set_fsai()
        x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
        assert info["flags"] & 4
        res.append((to_np(x), iters, info))
        S.close()
        G.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    A = O.system_matrix(g, lam, r)
    exact = O.DirectSolver(A)(rhs)
    kappa = O.jacobi_condition_number(A)
    e = rel(res[0][0], exact)
    print(f"rel err {e:.2e}, kappa {kappa:.1f}, iterations {res[0][1].max()}")
    assert res[0][2]["rel_res_max"] <= tol
    assert e <= kappa * tol * 4
