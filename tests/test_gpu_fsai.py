"""GPU FSAI factor (pfe_set_fsai, through the C ABI) against the oracle's FSAI
(a classical factor of the learned factor's form, on the lower pattern of A),
and PCG with it against the oracle's preconditioned PCG.

The device computes the factor in FP64 from the FP64 weights, so an FP64
context matches the oracle to rounding (<= 1e-11 relative); an FP32 context
stores the same values rounded to float (<= 1e-6)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth
from oracle import classical as C
from oracle.learned import pcg_preconditioned
from gpu_helpers import banner, gpu_graph, oracle_graph, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


HERE = os.path.dirname(os.path.abspath(__file__))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def scaled_factor(g, A, G):
    """(Gt_ji per undirected edge (i < j, lexicographic), diag(Gt)) with
    Gt = G D_A^{1/2}: the layout pfe_get_factor returns."""
    dA = A.diagonal()
    G = G.tocsr()
    ev = np.asarray(G[g.ej, g.ei]).ravel() * np.sqrt(dA[g.ei])
    return ev, G.diagonal() * np.sqrt(dA)


def case(name):
    if name == "ragged37x41_8":
        return synth.grid_workload(name, 37, 41, 4, 0.05, 11, gradient=0.2, stencil=8, d=6, n_inner=3, n_outer=2)
    return synth.make_workload(name, 0)


CASES = ["voronoi96x80_8nbr", "voronoi48x40_r2", "voronoi64_4nbr", "ragged37x41_8"]


def solver(wl, lam, r, fp64, strips="1", monkeypatch=None, tol=1e-10):
    from paper_1612_06496_amd import Solver
    if monkeypatch is not None:
        monkeypatch.setenv("PFE_STRIPS", strips)
    return Solver(gpu_graph(wl), wl.y0, lam=lam, r=r, n_inner=2, tol=tol, maxit=5000, fp64=fp64, persistent=False)


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("name", CASES)
def test_fsai_factor_matches_oracle(name, fp64):
    wl = case(name)
    banner(f"FSAI factor {name} fp64={fp64}")
    g = oracle_graph(wl)
    lam, r = 60.0, 0.5
    A = O.system_matrix(g, lam, r).tocsr()
    ev_o, dg_o = scaled_factor(g, A, C.fsai(A))
    S = solver(wl, lam, r, fp64)
    S.set_fsai()
    ev, dg = S.get_factor()
    e1, e2 = rel(to_np(ev), ev_o), rel(to_np(dg), dg_o)
    bound = 1e-11 if fp64 else 1e-6
    print(f"edge values rel {e1:.2e}, diagonal rel {e2:.2e} (bound {bound})")
    assert e1 <= bound and e2 <= bound


@pytest.mark.parametrize("strips", ["1", "0"])
@pytest.mark.parametrize("name", ["voronoi96x80_8nbr", "voronoi48x40_r2"])
def test_fsai_pcg_matches_oracle(name, strips, monkeypatch):
    """FP64 PCG with the FSAI factor: per-column iteration counts within one of
    the oracle's FSAI-PCG, and the direct solution within the condition-number
    bound; on image strips and on row chunks."""
    wl = case(name)
    banner(f"FSAI PCG {name} strips={strips}")
    g = oracle_graph(wl)
    lam, r, tol = 200.0, 1.0, 1e-10
    A = O.system_matrix(g, lam, r).tocsr()
    rhs = np.random.default_rng(7).normal(size=(g.n, wl.d))
    x0 = np.zeros_like(rhs)
    S = solver(wl, lam, r, True, strips, monkeypatch, tol=tol)
    S.set_fsai()
    x, iters, info = S.pcg(rhs, x0)
    _, it_o = pcg_preconditioned(A, rhs, x0, C.fsai_apply(C.fsai(A)), tol, 5000)
    _, it_j = pcg_preconditioned(A, rhs, x0, lambda v: v / A.diagonal()[:, None], tol, 5000)
    exact = O.DirectSolver(A)(rhs)
    e = rel(to_np(x), exact)
    kappa = O.jacobi_condition_number(A)
    print(f"iterations GPU {iters.tolist()} oracle {it_o.tolist()} (Jacobi {it_j.tolist()}); "
          f"rel err {e:.2e}; strips used {bool(info['flags'] & 2)}")
    assert np.all(np.abs(iters - it_o) <= 1)
    assert e <= kappa * tol * 4
    assert bool(info["flags"] & 2) == (strips == "1")


def test_fsai_batch_equals_solo():
    from paper_1612_06496_amd import Graph, Solver
    wls = synth.make_batch("voronoi_batch5_8nbr")
    banner("FSAI factor: batch == solo")
    parts = [gpu_graph(w) for w in wls]
    U = Graph.union(parts)
    kw = dict(lam=40.0, r=1.0, n_inner=2, tol=1e-8, maxit=2000, fp64=True, persistent=False)
    Sb = Solver(U, np.concatenate([w.y0 for w in wls]), **kw)
    Sb.set_fsai()
    ev, dg = (to_np(t) for t in Sb.get_factor())
    row0, e0 = U.segments
    for k, (w, p) in enumerate(zip(wls, parts)):
        Ss = Solver(p, w.y0, **kw)
        Ss.set_fsai()
        evs, dgs = (to_np(t) for t in Ss.get_factor())
        assert np.array_equal(ev[e0[k]:e0[k + 1]], evs)
        assert np.array_equal(dg[row0[k]:row0[k + 1]], dgs)


def test_fsai_needs_a_pixel_grid():
    from paper_1612_06496_amd import Solver
    from paper_1612_06496_amd._lib import PFEError
    wl = synth.edges_workload("gmm_small", 600, 8, 4, 6, 3, d=4, n_outer=1, n_inner=2)
    banner("FSAI on an edge-list graph is rejected")
    S = Solver(gpu_graph(wl), wl.y0, lam=10.0, r=1.0, n_inner=2, tol=1e-6, maxit=100, persistent=False)
    with pytest.raises(PFEError):
        S.set_fsai()


def test_fsai_window_graph_full_size_sampled_rows():
    """1024x1024, 5x5 window (d = 16, FP32 context as benchmarked): the factor
    on 300 sampled rows against the oracle's row-by-row FSAI."""
    wl = synth.make_workload("voronoi1024_r2", 0)
    banner("FSAI factor 1024x1024 window, sampled rows")
    g = oracle_graph(wl)
    lam, r = 100.0, 1.0
    A = O.system_matrix(g, lam, r).tocsr()
    S = solver(wl, lam, r, False, tol=1e-6)
    S.set_fsai()
    ev, dg = (to_np(t) for t in S.get_factor())
    dA = A.diagonal()
    # edge index of (j, i), j < i, in the lexicographic edge order
    key = g.ei.astype(np.int64) * g.n + g.ej
    rows = np.random.default_rng(11).choice(g.n, 300, replace=False)
    worst = 0.0
    for i in rows:
        Srow, gv = C.fsai_row(A, int(i))
        want = gv * np.sqrt(dA[Srow])
        got = np.empty_like(want)
        got[-1] = dg[i]
        lo = Srow[:-1].astype(np.int64)
        got[:-1] = ev[np.searchsorted(key, lo * g.n + i)]
        worst = max(worst, np.abs(got - want).max() / np.abs(want).max())
    print(f"worst sampled-row rel err {worst:.2e}")
    assert worst <= 1e-6


def test_full_size_counts_match_stored_oracle_counts():
    """1024x1024 window graph, first inner solve of a run (rhs = r/2 D Y0,
    x0 = Y0), FP32 PCG to 1e-6 with Jacobi and with FSAI at lambda/r = 1, 10,
    100, 1000: per-column iteration counts against the oracle's FP64 counts
    stored by tests/golden/make_preconditioner_counts.py, within 2 or 3 %
    (FP32 rounding can move the last iterations)."""
    from paper_1612_06496_amd import Solver
    with open(os.path.join(HERE, "golden", "preconditioner_counts_voronoi1024_r2.json")) as f:
        ref = json.load(f)
    wl = synth.make_workload(ref["workload"], ref["seed"])
    banner("Jacobi and FSAI iteration counts at 1024x1024 vs stored oracle counts")
    g = oracle_graph(wl)
    Y = O.orthonormalize_init(g, wl.y0)
    G = gpu_graph(wl)
    c = ref["c"]
    for ratio, cnt in ref["ratios"].items():
        lam, r = float(ratio) * c, c
        S = Solver(G, Y, lam=lam, r=r, n_inner=wl.n_inner, tol=ref["tol"], maxit=5000, init_ortho=False,
                   persistent=False)
        rhs = 0.5 * r * g.D[:, None] * Y
        _, it_j, _ = S.pcg(rhs, Y)
        S.set_fsai()
        _, it_f, _ = S.pcg(rhs, Y)
        print(f"lambda/r {ratio}: Jacobi max {it_j.max()} (oracle {max(cnt['jacobi'])}), FSAI max {it_f.max()} "
              f"(oracle {max(cnt['fsai'])}), IC(0) oracle {max(cnt['ic0'])}")
        for got, want in ((it_j, cnt["jacobi"]), (it_f, cnt["fsai"])):
            want = np.asarray(want)
            assert np.all(np.abs(got - want) <= np.maximum(2, 0.03 * want)), (ratio, got, want)
        del S


def test_soc_iteration_with_fsai_matches_oracle():
    """A SOC iteration whose solves use the FSAI factor (FP64, PCG to 1e-12)
    equals the oracle's (direct solves): the preconditioner changes the
    iteration counts, not the result."""
    from gpu_helpers import mid_run_state, penalties
    wl = case("voronoi48x40_r2")
    banner("SOC iteration with FSAI vs oracle")
    g = oracle_graph(wl)
    lam, r = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    solve, Y, P, B, _, _ = mid_run_state(g, wl, lam, r, 1, 0)
    Y1, P1, B1 = O.soc_outer_step(g, solve, Y, P, B, lam, r, wl.n_inner)
    from paper_1612_06496_amd import Solver
    S = Solver(gpu_graph(wl), Y, lam=lam, r=r, n_inner=wl.n_inner, tol=1e-12, maxit=3000, fp64=True,
               init_ortho=False, persistent=True)
    S.set("Y", Y); S.set("P", P); S.set("B", B)
    S.set_fsai()
    info = S.step("outer", info=True)
    eY, eP = rel(to_np(S.get("Y")), Y1), rel(to_np(S.get("P")), P1)
    print(f"Y {eY:.2e} P {eP:.2e}; CG iterations {info['cg_iters_total']}; workgroups {info['workgroups']}")
    assert eY <= 1e-9 and eP <= 1e-9
    assert info["workgroups"] == 0     # factor preconditioners run one launch per phase
