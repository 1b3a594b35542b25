"""Full-size parity in the launch shapes the benchmark times, against the FP64
oracle (Eq. 13 solved by the oracle's own CG to 1e-12, Eqs. 9-10, the polar
P-update of Algorithm 1).

1024 x 1024 Voronoi image, 5x5 window graph (24 slots, 12,552,210 edges),
d = 16, FP32 vectors: one SOC iteration with two Split-Bregman iterations
(every kernel of the one-launch-per-phase path runs: strip residual, strip CG
iterations, the 24-slot edge update and next right-hand side, the Gram and
apply passes) in the strip shapes sized for one and for two waves; Y, P, B
and the split variable b against the oracle, by relative Frobenius norm and
element-wise per column.  The learned factor on the same graph against the
oracle's network (bf16 products emulated) on every row."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, gpu_graph, maxrel, oracle_graph, rel
from oracle import learned as LN

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

WL = "voronoi1024_r2"
N_INNER = 2


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def window_case():
    wl = synth.make_workload(WL, 0)
    g = oracle_graph(wl)
    Y0 = O.orthonormalize_init(g, wl.y0)
    c = O.shrink_active_scale(g, Y0)
    solve = O.CGSolver(O.system_matrix(g, c, c), tol=1e-12)
    P0 = np.sqrt(g.D)[:, None] * Y0
    Y1, P1, B1, b1, _ = O.soc_outer_step(g, solve, Y0, P0, np.zeros_like(Y0), c, c, N_INNER, return_split=True)
    return wl, g, Y0, c, (Y1, P1, B1, b1)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("waves", [1, 2])
def test_window1024_soc_iteration_on_strips_vs_oracle(window_case, waves):
    from paper_1612_06496_amd import Solver
    wl, g, Y0, c, (Y1, P1, B1, b1) = window_case
    banner(f"1024x1024 window graph, d = 16, strips for {waves} wave(s): one SOC iteration vs oracle")
    G = gpu_graph(wl)
    S = Solver(G, Y0.astype(np.float32), lam=c, r=c, n_inner=N_INNER, tol=1e-6, maxit=1000, init_ortho=False,
               persistent=False, graphs=True)
    S.set_launch_shape(persistent=False, strips=waves)
    # the inner iterations one call each, so that b can be read before the
    # P-update closes the SOC iteration (b restarts from zero after it)
    S.step("inner")
    info = S.step("inner", info=True)
    assert info["flags"] & 2, info
    got_b = to_np(S.get("b"))
    S.step("outer")
    errs = {"b": (rel(got_b, b1), maxrel(got_b, b1))}
    got = {}
    for name, ref in (("Y", Y1), ("P", P1), ("B", B1)):
        got[name] = to_np(S.get(name))
        errs[name] = (rel(got[name], ref), maxrel(got[name], ref))
    # b = clamp(t, -1/lambda, 1/lambda) with t = w (y_i - y_j) + b_old (Eqs. 9-10)
    # and w <= 1: over the two inner iterations an error in Y moves b by at most
    # 2 max|dY| per iteration, so max|db| <= 4 max|dY| (twice that as margin for
    # the first solve's Y, which is not compared), plus FP32 rounding at the
    # threshold 1/lambda
    db = np.abs(got_b - b1).max()
    dY = np.abs(got["Y"] - Y1).max()
    bound_b = 8.0 * dY + 1e-6 / c
    print("errors (Frobenius, element-wise):", {k: f"{a:.2e}, {m:.2e}" for k, (a, m) in errs.items()},
          f"max|db| {db:.2e} (bound from max|dY| {bound_b:.2e}); CG iterations in the second solve "
          f"{info['cg_iters_total']}")
    for name in ("Y", "P"):
        assert errs[name][0] <= 2e-5 and errs[name][1] <= 1e-4, name
    # B = Z - P is a small difference of O(1) quantities
    assert errs["B"][0] <= 1e-3
    assert errs["b"][0] <= 1e-4 and db <= bound_b
    S.close()
    G.close()


@pytest.mark.timeout(900)
def test_window1024_soc_iteration_per_row_vs_oracle(window_case):
    """The launch shape the benchmark times on this graph: Jacobi PCG by per-row
    kernels (one workgroup per CU), the SOC iteration in one call, so that the
    first inner step's edge update also forms the second solve's residual.  Y
    and P against the oracle by Frobenius norm and element-wise, B relative to
    its norm."""
    from paper_1612_06496_amd import Solver
    wl, g, Y0, c, (Y1, P1, B1, _) = window_case
    banner("1024x1024 window graph, d = 16, per-row launches: one SOC iteration vs oracle")
    G = gpu_graph(wl)
    S = Solver(G, Y0.astype(np.float32), lam=c, r=c, n_inner=N_INNER, tol=1e-6, maxit=1000, init_ortho=False,
               persistent=False, graphs=True)
    S.set_launch_shape(persistent=False, pixel=1)
    info = S.solve(1, info=True)
    assert info["flags"] & 4 and info["flags"] & 8, info
    got = {k: to_np(S.get(k)) for k in ("Y", "P", "B")}
    errs = {k: (rel(got[k], ref), maxrel(got[k], ref)) for k, ref in (("Y", Y1), ("P", P1), ("B", B1))}
    print("errors (Frobenius, element-wise):", {k: f"{a:.2e}, {m:.2e}" for k, (a, m) in errs.items()},
          f"CG iterations {info['cg_iters_total']}")
    for name in ("Y", "P"):
        assert errs[name][0] <= 2e-5 and errs[name][1] <= 1e-4, name
    assert errs["B"][0] <= 1e-3
    S.close()
    G.close()


@pytest.mark.timeout(900)
def test_window1024_learned_factor_vs_oracle(window_case):
    from paper_1612_06496_amd import Mpnn, Solver
    wl, g, Y0, c, _ = window_case
    banner("1024x1024 window graph: learned factor vs oracle on every row")
    th = np.random.default_rng(11).normal(0.0, 0.2, size=LN.NPARAM)
    th[LN.NPARAM - 1] = LN.SOFTPLUS_ONE
    th = th.astype(np.float32).astype(np.float64)
    G = gpu_graph(wl)
    S = Solver(G, Y0.astype(np.float32), lam=10.0 * c, r=c, n_inner=1, init_ortho=False, persistent=False)
    net = Mpnn(th)
    S.set_learned(net)
    ev, dg = (to_np(t) for t in S.get_factor())
    SS = LN.ScaledSystem(g, 10.0 * c, c)
    gv, dgo = LN.factor(th, SS, bf16=True)
    up = SS.si < SS.sj                       # one slot per undirected edge, lexicographic
    ev_o, dg_o = gv.numpy()[up], dgo.numpy()
    e1 = np.abs(ev - ev_o).max() / np.abs(ev_o).max()
    e2 = np.abs(dg - dg_o).max() / np.abs(dg_o).max()
    print(f"factor at 1024^2: edge max rel {e1:.2e}, diagonal max rel {e2:.2e}")
    assert e1 <= 1e-2 and e2 <= 1e-2
    net.close()
    S.close()
    G.close()


@pytest.fixture(scope="module")
def knn200k_case():
    """The data-clustering workload's graph family at 200,000 points and its
    oracle SOC iteration (two Split-Bregman iterations, CG to 1e-12)."""
    wl = synth.make_edges_workload("gmm200k_knn16_rcm", 0)
    src, dst, dist2 = (t.cpu().numpy() for t in (wl.src, wl.dst, wl.dist2))
    g = O.build_edge_graph(wl.n, src, dst, dist2, wl.sigma)
    Y0 = O.orthonormalize_init(g, wl.y0)
    c = O.shrink_active_scale(g, Y0)
    solve = O.CGSolver(O.system_matrix(g, c, c), tol=1e-12)
    Y1, P1, _ = O.soc_outer_step(g, solve, Y0, np.sqrt(g.D)[:, None] * Y0, np.zeros_like(Y0), c, c, 2)
    return wl, Y0, c, Y1, P1


@pytest.mark.timeout(900)
@pytest.mark.parametrize("shape", ["autotuned", "per-row", "per-row-2"])
def test_knn200k_soc_iteration_vs_oracle(knn200k_case, shape):
    """The data-clustering workload's graph family at 200,000 points (Gaussian
    mixture in R^32, symmetrised exact 16-NN graph in reverse Cuthill-McKee
    order, d = 20; general CSR slot layout): one SOC iteration with two
    Split-Bregman iterations in the autotuned launch shape and in per-row
    launches (one and two workgroups per CU) against the oracle (CG to 1e-12),
    by Frobenius norm and element-wise per column."""
    from paper_1612_06496_amd import Graph, Solver
    banner(f"200k-point k-NN graph, d = 20: one SOC iteration vs oracle ({shape})")
    wl, Y0, c, Y1, P1 = knn200k_case
    G = Graph.edges(wl.n, wl.src, wl.dst, wl.dist2, wl.sigma)
    S = Solver(G, Y0.astype(np.float32), lam=c, r=c, n_inner=2, tol=1e-6, maxit=1000, init_ortho=False)
    if shape == "autotuned":
        shapes = S.autotune(1)
        chosen = [s_ for s_ in shapes if s_["chosen"]][0]
    else:
        wpc = 2 if shape == "per-row-2" else 1
        S.set_launch_shape(persistent=False, pixel=wpc)
        chosen = f"per-row launches, {wpc} workgroup(s) per CU"
    info = S.solve(1, info=True)
    if shape != "autotuned":
        assert info["flags"] & 4
    Yg, Pg = to_np(S.get("Y")), to_np(S.get("P"))
    eY, eP = rel(Yg, Y1), rel(Pg, P1)
    mY, mP = maxrel(Yg, Y1), maxrel(Pg, P1)
    print(f"Y {eY:.2e} ({mY:.2e} element-wise) P {eP:.2e} ({mP:.2e}); shape {chosen}; "
          f"CG iterations per solve {info['cg_iters_total'] / info['solves']:.2f}")
    assert eY <= 2e-5 and eP <= 2e-5
    assert mY <= 1e-4 and mP <= 1e-4
    S.close()
    G.close()
