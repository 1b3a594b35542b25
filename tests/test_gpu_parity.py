"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Bounds are the ones the solver's precision supports:
FP32 vectors with a PCG stopped at relative residual 1e-6 give per-step
relative errors <= 1e-5; the FP64 instantiation reaches the oracle to ~1e-10
when its PCG tolerance is tight."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, gpu_graph, maxrel, mid_run_state, oracle_graph, penalties, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def small_edges_workload(n=900, d=5, seed=3):
    return synth.edges_workload("gmm_small", n, 8, 4, 6, seed, d=d, n_outer=3, n_inner=3)


GRAPH_CASES = ["voronoi64_4nbr", "voronoi96x80_8nbr", "voronoi48x40_r2", "edges"]


def load(name, seed=0):
    if name == "edges":
        return small_edges_workload()
    return synth.make_workload(name, seed)


# --- graph build -------------------------------------------------------------

@pytest.mark.parametrize("name", GRAPH_CASES)
def test_graph_build_matches_oracle(name):
    banner(f"graph build {name}")
    wl = load(name)
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    csr = G.csr()
    assert G.n == g.n and G.n_edges == g.n_edges
    Wo = g.adjacency().tocsr()
    Wo.sort_indices()
    assert np.array_equal(csr["rowptr"].cpu().numpy(), Wo.indptr)
    assert np.array_equal(csr["col"].cpu().numpy(), Wo.indices)
    w_gpu = csr["w"].cpu().numpy()
    w_ref = Wo.data.astype(np.float32)
    # both evaluate the heat kernel in FP64 and round to FP32: at most 1 ulp apart
    ulp = np.abs(w_gpu.view(np.int32).astype(np.int64) - w_ref.view(np.int32).astype(np.int64))
    assert ulp.max() <= 1, ulp.max()
    deg = csr["degree"].cpu().numpy()
    assert np.abs(deg - g.D).max() <= 1e-13 * g.D.max()


def test_graph_errors_are_reported():
    from paper_1612_06496_amd import Graph
    from paper_1612_06496_amd._lib import PFEError, PFE_E_GRAPH
    banner("graph errors")
    # isolated vertex 3
    with pytest.raises(PFEError) as e:
        Graph.edges(4, np.array([0, 1]), np.array([1, 2]), np.array([0.1, 0.2]), 1.0)
    assert e.value.status == PFE_E_GRAPH
    # self loop, duplicate, out of range
    for src, dst in (([0, 1, 2], [1, 2, 2]), ([0, 1, 1, 2], [1, 2, 2, 3]), ([0, 1, 5], [1, 2, 3])):
        with pytest.raises(PFEError) as e:
            Graph.edges(4, np.array(src), np.array(dst), np.full(len(src), 0.1), 1.0)
        assert e.value.status == PFE_E_GRAPH
    # non-finite feature -> non-finite weight
    feat = np.random.default_rng(0).uniform(size=(6 * 5, 3)).astype(np.float32)
    feat[7, 1] = np.nan
    with pytest.raises(PFEError) as e:
        Graph.grid(feat, 6, 5, 4, 0.1)
    assert e.value.status == PFE_E_GRAPH


# --- operator and solver -------------------------------------------------------

@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("name", ["voronoi96x80_8nbr", "voronoi48x40_r2", "edges"])
def test_apply_A_matches_oracle(name, fp64):
    from paper_1612_06496_amd import Solver
    banner(f"apply_A {name} fp64={fp64}")
    wl = load(name)
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    lam, r = 3.0, 0.7
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=2, fp64=fp64, persistent=False)
    X = np.random.default_rng(1).normal(size=(g.n, wl.d))
    if not fp64:
        X = X.astype(np.float32).astype(np.float64)
    Q = to_np(S.apply_A(X))
    Qo = O.system_matrix(g, lam, r) @ X
    err = np.abs(Q - Qo).max() / np.abs(Qo).max()
    print(f"apply_A max rel err {err:.3e}")
    assert err <= (1e-14 if fp64 else 2e-6)


@pytest.mark.parametrize("fp64", [False, True])
def test_pcg_matches_direct_solve(fp64):
    from paper_1612_06496_amd import Solver
    banner(f"pcg fp64={fp64}")
    wl = load("voronoi96x80_8nbr")
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    for lam, r in ((1.0, 1.0), (20.0, 1.0)):
        tol = 1e-12 if fp64 else 1e-6
        S = Solver(G, wl.y0, lam=lam, r=r, n_inner=2, tol=tol, maxit=2000, fp64=fp64, persistent=False)
        A = O.system_matrix(g, lam, r)
        rhs = np.random.default_rng(2).normal(size=(g.n, wl.d))
        x, iters, info = S.pcg(rhs, np.zeros_like(rhs))
        exact = O.DirectSolver(A)(rhs)
        kappa = O.jacobi_condition_number(A) if g.n <= 8000 else 100.0
        err = rel(to_np(x), exact)
        print(f"lam/r={lam/r} kappa={kappa:.1f} iters={iters.max()} rel err={err:.2e} bound={kappa*tol*4:.2e}")
        assert info["rel_res_max"] <= tol
        assert err <= kappa * tol * 4 + (0 if fp64 else 1e-6)
        # same iteration counts as the oracle's own Jacobi-PCG, within one
        _, it_o, _ = O.pcg(A, rhs, np.zeros_like(rhs), 1.0 / A.diagonal(), tol, 2000)
        assert np.all(np.abs(iters - it_o) <= (1 if fp64 else 3))


def test_pcg_zero_rhs_column_and_noconv():
    from paper_1612_06496_amd import Solver
    from paper_1612_06496_amd._lib import PFEError, PFE_E_NOCONV
    banner("pcg zero column / maxit")
    wl = load("voronoi48x40_r2")
    G = gpu_graph(wl)
    S = Solver(G, wl.y0, lam=10.0, r=1.0, n_inner=2, tol=1e-6, maxit=1, persistent=False)
    rhs = np.random.default_rng(3).normal(size=(G.n, wl.d)).astype(np.float32)
    rhs[:, 2] = 0.0
    x0 = np.ones_like(rhs)
    with pytest.raises(PFEError) as e:
        S.pcg(rhs, x0)
    assert e.value.status == PFE_E_NOCONV
    x, iters, info = S.pcg(rhs, x0, allow_noconv=True)
    assert np.all(to_np(x)[:, 2] == 0.0) and iters[2] == 0
    assert iters.max() == 1


# --- inner and outer steps from an injected oracle state ------------------------

STEP_CASES = [("voronoi96x80_8nbr", False), ("voronoi64_4nbr", True), ("edges", False)]


@pytest.mark.parametrize("k_in", [1, 2])
@pytest.mark.parametrize("name,fp64", STEP_CASES)
def test_inner_step_parity(name, fp64, k_in):
    """One Split-Bregman iteration from an injected oracle state at inner
    index 1 or 2 (the two parities of the double-buffered split variable)."""
    from paper_1612_06496_amd import Solver
    banner(f"inner step {name} fp64={fp64} inner index {k_in}")
    wl = load(name)
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    lam, r = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    solve, Y, P, B, b, dd = mid_run_state(g, wl, lam, r, 1, k_in)
    tol = 1e-12 if fp64 else 1e-6
    S = Solver(G, Y, lam=lam, r=r, n_inner=wl.n_inner, tol=tol, maxit=2000, fp64=fp64,
               keep_split=True, init_ortho=False, persistent=False)
    S.set("Y", Y); S.set("P", P); S.set("B", B)
    S.inner_index = k_in
    S.set("b", b); S.set("d", dd)
    # the stored right-hand side equals Eq. 13's
    rhs_o = O.sb_rhs(g, P, B, b, dd, lam, r)
    e_rhs = rel(to_np(S.get("rhs")), rhs_o)
    info = S.step("inner", info=True)
    Y1, b1, dd1 = O.sb_inner_step(g, solve, Y, P, B, b, dd, lam, r)
    eY = rel(to_np(S.get("Y")), Y1)
    t = g.M @ Y1 + b
    eb = np.linalg.norm(to_np(S.get("b")) - b1) / np.linalg.norm(t)
    ed = np.linalg.norm(to_np(S.get("d")) - dd1) / np.linalg.norm(t)
    frac = np.mean(dd1 != 0)
    bound = 1e-10 if fp64 else 1e-5
    print(f"rhs {e_rhs:.2e} Y {eY:.2e} b {eb:.2e} d {ed:.2e} (bound {bound}); "
          f"cg iters {info['cg_iters_max']}; nonzero d fraction {frac:.4f}")
    assert e_rhs <= (1e-13 if fp64 else 1e-6)
    assert eY <= bound and eb <= bound and ed <= bound
    if wl.lam is None:
        assert frac > 0.0      # the shrink is active
    # monitor: nonzero fraction of the stored d (entries with |t| at the
    # threshold may fall either way in FP32)
    nz = S.monitor()["split_nonzero"]
    print(f"nonzero d fraction: GPU monitor {nz:.5f}, oracle {frac:.5f}")
    assert abs(nz - frac) <= (1e-12 if fp64 else 1e-3)


@pytest.mark.parametrize("name,fp64", STEP_CASES)
@pytest.mark.parametrize("ortho", ["polar", "chol"])
def test_outer_step_parity(name, fp64, ortho):
    from paper_1612_06496_amd import Solver
    banner(f"outer step {name} fp64={fp64} {ortho}")
    wl = load(name)
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    lam, r = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    solve, Y, P, B, _, _ = mid_run_state(g, wl, lam, r, 2, 0)
    tol = 1e-12 if fp64 else 1e-6
    S = Solver(G, Y, lam=lam, r=r, n_inner=wl.n_inner, tol=tol, maxit=2000, fp64=fp64, ortho=ortho,
               init_ortho=False, persistent=False)
    S.set("Y", Y); S.set("P", P); S.set("B", B)
    S.step("outer")
    Y1, P1, B1 = O.soc_outer_step(g, solve, Y, P, B, lam, r, wl.n_inner, ortho)
    eY, eP = rel(to_np(S.get("Y")), Y1), rel(to_np(S.get("P")), P1)
    eB = np.linalg.norm(to_np(S.get("B")) - B1) / np.linalg.norm(P1)
    bound = 1e-9 if fp64 else 1e-5
    print(f"Y {eY:.2e} P {eP:.2e} B/|P| {eB:.2e} bound {bound}")
    assert eY <= bound and eP <= bound and eB <= bound
    m = S.monitor()
    assert m["orthogonality"] <= (1e-12 if fp64 else 1e-5)
    assert m["split_nonzero"] == -1.0          # d is not stored without keep_split


# --- end to end ------------------------------------------------------------------

@pytest.mark.parametrize("persistent", [False, True])
def test_end_to_end_fp64_small_image(persistent):
    """64x64, 4-neighbour, d = 4, lambda = r = 1, 10 x 5 iterations in FP64."""
    from paper_1612_06496_amd import Solver
    banner(f"end-to-end voronoi64_4nbr fp64 persistent={persistent}")
    wl = load("voronoi64_4nbr")
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    Y0, _ = O.le_init(g, wl.d)
    ref = O.pfe_run(g, Y0, wl.lam, wl.r, wl.n_outer, wl.n_inner)
    S = Solver(G, Y0, lam=wl.lam, r=wl.r, n_inner=wl.n_inner, tol=1e-12, maxit=2000, fp64=True,
               persistent=persistent)
    info = S.solve(wl.n_outer, info=True)
    yh = to_np(S.get("Yhat"))
    yh_ref = ref.yhat(g)
    f, f_ref = O.objective(g, yh), O.objective(g, yh_ref)
    # |f(y) - f(y')| <= ||M (y - y')||_1 by the triangle inequality
    bound = float(np.abs(g.M @ (yh - yh_ref)).sum()) * (1 + 1e-9) + 1e-300
    print(f"objective {f:.6e} vs {f_ref:.6e} (|diff| {abs(f - f_ref):.2e}, bound {bound:.2e}); "
          f"Yhat rel {rel(yh, yh_ref):.2e}; iters {info}")
    assert abs(f - f_ref) <= bound
    assert abs(f - f_ref) <= 1e-3 * f_ref
    assert rel(yh, yh_ref) <= 1e-8
    assert O.constraint_residual(g, yh) <= 1e-10
    agree, _ = O.kmeans_agreement(yh_ref, yh, wl.n_clusters)
    assert agree >= 0.99


@pytest.mark.parametrize("persistent", [False, True])
def test_end_to_end_fp32_small_image(persistent):
    from paper_1612_06496_amd import Solver
    banner(f"end-to-end voronoi96x80_8nbr fp32 persistent={persistent}")
    wl = load("voronoi96x80_8nbr")
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    Y0 = O.orthonormalize_init(g, wl.y0)
    lam, r = penalties(wl, g, Y0)
    ref = O.pfe_run(g, wl.y0, lam, r, wl.n_outer, wl.n_inner)
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=wl.n_inner, tol=wl.tol, maxit=1000,
               persistent=persistent)
    info = S.solve(wl.n_outer, info=True)
    yh = to_np(S.get("Yhat"))
    yh_ref = ref.yhat(g)
    f, f_ref = O.objective(g, yh), O.objective(g, yh_ref)
    m = S.monitor()
    print(f"objective {f:.6e} vs {f_ref:.6e} (gpu monitor {m['objective']:.6e}); "
          f"constraint {O.constraint_residual(g, yh):.2e}; info {info}")
    assert abs(f - f_ref) <= 1e-3 * f_ref
    assert abs(m["objective"] - f) <= 1e-5 * f
    assert O.constraint_residual(g, yh) <= 1e-5
    assert m["constraint"] <= 1e-5
    agree, _ = O.kmeans_agreement(yh_ref, yh, wl.n_clusters)
    assert agree >= 0.99


def test_persistent_equals_multi_launch():
    from paper_1612_06496_amd import Solver
    banner("persistent vs multi-launch")
    wl = load("voronoi96x80_8nbr")
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    lam, r = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    out = []
    for persistent in (False, True):
        S = Solver(G, wl.y0, lam=lam, r=r, n_inner=wl.n_inner, tol=1e-6, persistent=persistent)
        S.solve(2)
        out.append(to_np(S.get("P")))
    print("rel diff", rel(out[0], out[1]))
    assert rel(out[0], out[1]) <= 1e-5


def test_determinism_bitwise():
    from paper_1612_06496_amd import Solver
    banner("determinism")
    wl = load("voronoi96x80_8nbr")
    G = gpu_graph(wl)
    res = []
    for _ in range(2):
        S = Solver(G, wl.y0, lam=50.0, r=50.0, n_inner=3, tol=1e-6, persistent=True)
        S.solve(2)
        res.append(S.get("P").cpu().numpy())
    assert np.array_equal(res[0], res[1])


def test_checkpoint_resume_bitwise():
    """2 SOC iterations, save (Y, P, B), restore in a new context, 2 more ==
    4 in one go."""
    from paper_1612_06496_amd import Solver
    banner("checkpoint / resume")
    wl = load("voronoi96x80_8nbr")
    G = gpu_graph(wl)
    kw = dict(lam=50.0, r=50.0, n_inner=3, tol=1e-6, persistent=True)
    S = Solver(G, wl.y0, **kw)
    S.solve(4)
    ref = S.get("P").cpu().numpy()
    S1 = Solver(G, wl.y0, **kw)
    S1.solve(2)
    state = {k: S1.get(k) for k in ("Y", "P", "B")}
    S2 = Solver(G, state["Y"], init_ortho=False, **kw)
    for k, v in state.items():
        S2.set(k, v)
    S2.solve(2)
    assert np.array_equal(S2.get("P").cpu().numpy(), ref)


# --- edge cases ---------------------------------------------------------------------

def test_rank_deficient_init_is_rejected():
    from paper_1612_06496_amd import Solver
    from paper_1612_06496_amd._lib import PFEError, PFE_E_RANK
    banner("rank-deficient Y0")
    wl = load("voronoi48x40_r2")
    G = gpu_graph(wl)
    Y0 = wl.y0.copy()
    Y0[:, 3] = Y0[:, 1]
    with pytest.raises(PFEError) as e:
        Solver(G, Y0, lam=1.0, r=1.0, n_inner=2)
    assert e.value.status == PFE_E_RANK


@pytest.mark.parametrize("d", [1, 3, 5, 25, 32])
def test_dimensions_and_ragged_sizes(d):
    """d = 1 and d = 32, and an image whose pixel count is not a multiple of
    the rows handled per pass, against the oracle."""
    from paper_1612_06496_amd import Solver
    banner(f"dimension d={d}")
    wl = synth.grid_workload("ragged", 37, 41, 5, 0.05, 9, stencil=8, d=d, n_outer=2, n_inner=2)
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    lam, r = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    ref = O.pfe_run(g, wl.y0, lam, r, 2, 2)
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=2, tol=1e-12, maxit=3000, fp64=True, persistent=True)
    S.solve(2)
    e = rel(to_np(S.get("P")), ref.P)
    print(f"d={d} P rel err {e:.2e}")
    assert e <= 1e-9


def test_edge_quantile_matches_order_statistic():
    from paper_1612_06496_amd import Solver
    banner("edge quantile")
    wl = load("voronoi96x80_8nbr")
    g = oracle_graph(wl)
    G = gpu_graph(wl)
    S = Solver(G, wl.y0, lam=1.0, r=1.0, n_inner=2, fp64=True)
    Y = to_np(S.get("Y"))
    v = np.sort(np.abs(g.M @ Y).reshape(-1))
    for q in (0.5, 0.99, 1.0):
        got = S.edge_quantile(q)
        want = v[int(np.floor(q * (v.size - 1)))]
        assert abs(got - want) <= 1e-9 * want
    S32 = Solver(G, wl.y0, lam=1.0, r=1.0, n_inner=2)
    got = S32.edge_quantile(0.99)
    assert abs(got - v[int(np.floor(0.99 * (v.size - 1)))]) <= 1e-5 * got


@pytest.mark.parametrize("name", ["voronoi96x80_8nbr", "voronoi48x40_r2", "voronoi64_4nbr"])
def test_lds_row_cache_is_bitwise_neutral(name, monkeypatch):
    """The persistent kernel's LDS copy of the rows' slot data gives bitwise the
    same iteration as reading it from global memory."""
    from paper_1612_06496_amd import Solver
    banner(f"LDS row cache {name}")
    wl = load(name)
    G = gpu_graph(wl)
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("PFE_ROWCACHE", flag)
        S = Solver(G, wl.y0, lam=30.0, r=30.0, n_inner=3, tol=1e-6, maxit=1000, persistent=True)
        info = S.solve(2, info=True)
        assert info["workgroups"] > 0
        out.append((to_np(S.get("Y")), to_np(S.get("P")), to_np(S.get("B"))))
    for k in range(3):
        assert np.array_equal(out[0][k], out[1][k])


def test_graph_replay_is_bitwise_neutral():
    """One-launch-per-phase PCG replayed from HIP graphs (many replays across
    inner solves, with host synchronisation between them) gives bitwise the
    iteration of host-launched kernels."""
    from paper_1612_06496_amd import Solver
    banner("graph replay (Jacobi)")
    wl = load("voronoi96x80_8nbr")
    G = gpu_graph(wl)
    out = []
    for graphs in (True, False):
        S = Solver(G, wl.y0, lam=30.0, r=30.0, n_inner=3, tol=1e-6, maxit=1000, persistent=False, graphs=graphs)
        info = S.solve(2, info=True)
        out.append((to_np(S.get("Y")), to_np(S.get("P")), info["cg_iters_total"]))
    assert out[0][2] == out[1][2]
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_second_workgroup_weight_partition(monkeypatch):
    """Persistent, teams of one workgroup: giving the second workgroup placed
    on each CU a smaller share of the rows changes only which rows each
    workgroup owns, so one SOC iteration agrees with the equal split up to the
    summation order of the FP64 partials, and stays bitwise reproducible."""
    from paper_1612_06496_amd import Solver
    banner("second-workgroup row weight (481x321)")
    wl = load("voronoi481x321_8nbr")
    G = gpu_graph(wl)
    monkeypatch.setenv("PFE_TEAM", "1")
    out = []
    for w in ("1.0", "0.8", "0.8"):
        monkeypatch.setenv("PFE_SECOND_WEIGHT", w)
        S = Solver(G, wl.y0, lam=2000.0, r=2000.0, n_inner=3, tol=1e-6, maxit=1000, persistent=True)
        info = S.solve(1, info=True)
        assert info["workgroups"] > 0 and info["workgroups"] % 16 == 0
        out.append((to_np(S.get("Y")), to_np(S.get("P"))))
    e = max(rel(out[1][k], out[0][k]) for k in range(2))
    print(f"weighted vs equal rows: rel {e:.2e}")
    assert e <= 1e-5
    assert all(np.array_equal(out[1][k], out[2][k]) for k in range(2))


def test_headline_image_soc_iterations_vs_oracle():
    """481x321, d = 10, shrink-active penalties: two SOC iterations (10 inner
    solves each) in the launch shape the autotuner picks, as the benchmark runs
    them, against the oracle's direct solves; the GPU monitors against the
    oracle's objective and constraint."""
    from paper_1612_06496_amd import Solver
    wl = load("voronoi481x321_8nbr")
    banner("481x321 full size: 2 SOC iterations in the autotuned shape vs oracle")
    g = oracle_graph(wl)
    Y0 = O.orthonormalize_init(g, wl.y0)
    c = O.shrink_active_scale(g, Y0)
    ref = O.pfe_run(g, Y0, c, c, 2, wl.n_inner)
    S = Solver(gpu_graph(wl), Y0, lam=c, r=c, n_inner=wl.n_inner, tol=1e-6, maxit=1000, init_ortho=False)
    shapes = S.autotune(1)
    info = S.solve(2, info=True)
    Yg, Pg = to_np(S.get("Y")), to_np(S.get("P"))
    eY, eP = rel(Yg, ref.Y), rel(Pg, ref.P)
    mY, mP = maxrel(Yg, ref.Y), maxrel(Pg, ref.P)
    yh = ref.yhat(g)
    m = S.monitor()
    f_ref = O.objective(g, yh)
    chosen = [s for s in shapes if s["chosen"]][0]
    print(f"Y {eY:.2e} (element-wise {mY:.2e}) P {eP:.2e} (element-wise {mP:.2e}); objective "
          f"{m['objective']:.6e} vs {f_ref:.6e}; constraint {m['constraint']:.2e}; "
          f"shape {chosen}; CG iterations per solve {info['cg_iters_total'] / info['solves']:.2f}")
    assert eY <= 2e-5 and eP <= 2e-5
    assert mY <= 1e-4 and mP <= 1e-4
    assert abs(m["objective"] - f_ref) <= 1e-3 * f_ref
    assert m["constraint"] <= 1e-5
    assert O.constraint_residual(g, to_np(S.get("Yhat"))) <= 1e-5


@pytest.mark.parametrize("persistent", [True, False])
def test_lambda_zero_reduces_to_scaled_split_target(persistent):
    """lambda = 0 (no edge term, infinite shrink threshold): every inner solve
    gives Y = D^{-1/2} (P - B) exactly (Eq. 13 with A = r/2 D), so a SOC
    iteration from an oracle state with B != 0 equals the oracle's, in both
    launch shapes."""
    from paper_1612_06496_amd import Solver
    wl = load("voronoi96x80_8nbr")
    banner(f"lambda = 0, persistent={persistent}")
    g = oracle_graph(wl)
    lam0, r0 = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    solve, Y, P, B, _, _ = mid_run_state(g, wl, lam0, r0, 1, 0)
    r = r0
    S = Solver(gpu_graph(wl), Y, lam=0.0, r=r, n_inner=wl.n_inner, tol=1e-13, maxit=100, fp64=True,
               init_ortho=False, persistent=persistent)
    S.set("Y", Y); S.set("P", P); S.set("B", B)
    info = S.step("outer", info=True)
    target = (P - B) / np.sqrt(g.D)[:, None]
    Y1, P1, B1 = O.soc_outer_step(g, O.DirectSolver(O.system_matrix(g, 0.0, r)), Y, P, B, 0.0, r, wl.n_inner)
    eT = rel(to_np(S.get("Y")), target)
    eP = rel(to_np(S.get("P")), P1)
    print(f"Y vs D^-1/2 (P - B): {eT:.2e}; P vs oracle {eP:.2e}; CG iterations per solve "
          f"{info['cg_iters_total'] / info['solves']:.2f}")
    assert eT <= 1e-12 and eP <= 1e-12
    assert info["cg_iters_max"] <= 1
