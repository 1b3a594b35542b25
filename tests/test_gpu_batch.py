"""GPU batching: a block-diagonal union of uneven graphs, solved side by side
with per-graph CG scalars, convergence and P-update.  Each graph of the batch
must get what it gets alone (GPU vs GPU, only the summation order of the FP64
reductions differs) and what the FP64 oracle computes for it."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, gpu_graph, maxrel, oracle_graph, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

BATCH = "voronoi_batch5_8nbr"


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def build(wls):
    from paper_1612_06496_amd import Graph
    parts = [gpu_graph(w) for w in wls]
    return parts, Graph.union(parts)


def fixed_penalties(wls):
    """One lambda = r for the whole batch: the shrink-active scale of the first image."""
    g0 = oracle_graph(wls[0])
    c = O.shrink_active_scale(g0, O.orthonormalize_init(g0, wls[0].y0), 0.99)
    return c, c


def test_union_structure_is_block_diagonal():
    from paper_1612_06496_amd import Graph
    banner("graph union structure")
    wls = synth.make_batch(BATCH)
    parts, U = build(wls)
    row0, edge0 = U.segments
    assert np.array_equal(row0, np.cumsum([0] + [p.n for p in parts]))
    assert np.array_equal(edge0, np.cumsum([0] + [p.n_edges for p in parts]))
    cu = {k: v.cpu().numpy() for k, v in U.csr().items()}
    s0 = 0
    for k, p in enumerate(parts):
        cp = {kk: v.cpu().numpy() for kk, v in p.csr().items()}
        v0, v1 = row0[k], row0[k + 1]
        assert np.array_equal(cu["rowptr"][v0:v1 + 1] - s0, cp["rowptr"])
        sl = slice(cp["rowptr"][0] + s0, cp["rowptr"][-1] + s0)
        assert np.array_equal(cu["col"][sl] - v0, cp["col"])
        assert np.array_equal(cu["w"][sl], cp["w"])
        assert np.array_equal(cu["degree"][v0:v1], cp["degree"])
        s0 += cp["rowptr"][-1]
    # mixed stencils and an edge-list graph (general slot layout); unions nest
    edges = synth.edges_workload("gmm", 400, 8, 3, 5, 1, d=4)
    g4 = synth.grid_workload("g4", 20, 24, 4, 0.05, 5, stencil=4, d=4)
    mixed = [gpu_graph(edges), gpu_graph(g4), parts[0]]
    M = Graph.union([Graph.union(mixed[:2]), mixed[2]])
    r0, e0 = M.segments
    assert np.array_equal(r0, np.cumsum([0] + [p.n for p in mixed]))
    assert np.array_equal(e0, np.cumsum([0] + [p.n_edges for p in mixed]))
    cm = M.csr()
    deg = cm["degree"].cpu().numpy()
    ref = np.concatenate([p.csr()["degree"].cpu().numpy() for p in mixed])
    assert np.array_equal(deg, ref)


def test_union_errors():
    from paper_1612_06496_amd import Graph, Solver
    from paper_1612_06496_amd._lib import PFEError, PFE_E_ARG
    banner("graph union errors")
    with pytest.raises(PFEError) as e:
        Graph.union([])
    assert e.value.status == PFE_E_ARG
    # a part with no more vertices than d cannot carry a d-dimensional embedding
    big = synth.grid_workload("big", 20, 24, 4, 0.05, 1, stencil=8, d=6)
    tiny = synth.grid_workload("tiny", 2, 3, 2, 0.05, 2, stencil=8, d=6)
    U = Graph.union([gpu_graph(big), gpu_graph(tiny)])
    with pytest.raises(PFEError) as e:
        Solver(U, np.concatenate([big.y0, tiny.y0]), lam=1.0, r=1.0, n_inner=2)
    assert e.value.status == PFE_E_ARG


def test_rank_deficient_segment_is_rejected():
    from paper_1612_06496_amd import Solver
    from paper_1612_06496_amd._lib import PFEError, PFE_E_RANK
    banner("batch rank-deficient segment")
    wls = synth.make_batch(BATCH)
    parts, U = build(wls)
    Y0 = [w.y0.copy() for w in wls]
    Y0[2][:, 1] = Y0[2][:, 0]
    with pytest.raises(PFEError) as e:
        Solver(U, np.concatenate(Y0), lam=1.0, r=1.0, n_inner=2)
    assert e.value.status == PFE_E_RANK


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("persistent", [True, False])
def test_batch_matches_solo(fp64, persistent):
    from paper_1612_06496_amd import Solver
    banner(f"batch == solo fp64={fp64} persistent={persistent}")
    wls = synth.make_batch(BATCH)
    parts, U = build(wls)
    lam, r = fixed_penalties(wls)
    kw = dict(lam=lam, r=r, n_inner=wls[0].n_inner, tol=1e-11 if fp64 else 1e-6, maxit=3000, fp64=fp64,
              persistent=persistent)
    S = Solver(U, np.concatenate([w.y0 for w in wls]), **kw)
    info = S.solve(2, info=True)
    if persistent:
        assert info["workgroups"] > 0
    got = {k: to_np(S.get(k)) for k in ("Y", "P", "B")}
    row0, _ = U.segments
    worst = 0.0
    for k, (w, p) in enumerate(zip(wls, parts)):
        Ss = Solver(p, w.y0, **kw)
        Ss.solve(2)
        sl = slice(row0[k], row0[k + 1])
        eY = rel(got["Y"][sl], to_np(Ss.get("Y")))
        eP = rel(got["P"][sl], to_np(Ss.get("P")))
        eB = np.linalg.norm(got["B"][sl] - to_np(Ss.get("B"))) / np.linalg.norm(to_np(Ss.get("P")))
        worst = max(worst, eY, eP, eB)
    bound = 1e-8 if fp64 else 1e-5
    print(f"worst segment rel err {worst:.2e} (bound {bound}); info {info}")
    assert worst <= bound


def test_batch_outer_step_matches_oracle():
    """One SOC iteration of the batch in FP64 against the oracle's, graph by graph."""
    from paper_1612_06496_amd import Solver
    banner("batch outer step vs oracle")
    wls = synth.make_batch(BATCH)
    parts, U = build(wls)
    lam, r = fixed_penalties(wls)
    S = Solver(U, np.concatenate([w.y0 for w in wls]), lam=lam, r=r, n_inner=wls[0].n_inner, tol=1e-12,
               maxit=3000, fp64=True, persistent=True)
    S.solve(1)
    Yg, Pg = to_np(S.get("Y")), to_np(S.get("P"))
    row0, _ = U.segments
    worst = 0.0
    for k, w in enumerate(wls):
        g = oracle_graph(w)
        Y = O.orthonormalize_init(g, w.y0)
        P = np.sqrt(g.D)[:, None] * Y
        solve = O.DirectSolver(O.system_matrix(g, lam, r))
        Y1, P1, _ = O.soc_outer_step(g, solve, Y, P, np.zeros_like(Y), lam, r, w.n_inner)
        sl = slice(row0[k], row0[k + 1])
        worst = max(worst, rel(Yg[sl], Y1), rel(Pg[sl], P1))
    print(f"worst segment rel err vs oracle {worst:.2e}")
    assert worst <= 1e-9


def test_batch_monitor_is_per_segment():
    from paper_1612_06496_amd import Solver
    banner("batch monitor")
    wls = synth.make_batch(BATCH)
    parts, U = build(wls)
    lam, r = fixed_penalties(wls)
    kw = dict(lam=lam, r=r, n_inner=wls[0].n_inner, tol=1e-11, maxit=3000, fp64=True)
    S = Solver(U, np.concatenate([w.y0 for w in wls]), **kw)
    S.solve(2)
    m = S.monitor()
    f_solo = 0.0
    yh = to_np(S.get("Yhat"))
    row0, _ = U.segments
    for k, (w, p) in enumerate(zip(wls, parts)):
        Ss = Solver(p, w.y0, **kw)
        Ss.solve(2)
        f_solo += Ss.monitor()["objective"]
        g = oracle_graph(w)
        assert O.constraint_residual(g, yh[row0[k]:row0[k + 1]]) <= 1e-10
    print(f"batch monitor {m}; sum of solo objectives {f_solo:.12e}")
    assert abs(m["objective"] - f_solo) <= 1e-9 * f_solo
    assert m["constraint"] <= 1e-10 and m["orthogonality"] <= 1e-10


def test_batch_learned_factor_and_pcg():
    """The network's factor on a batch is each graph's own factor; learned PCG
    solves every segment."""
    from paper_1612_06496_amd import Mpnn, Solver
    banner("batch learned factor + PCG")
    wls = synth.make_batch(BATCH)
    parts, U = build(wls)
    th = np.random.default_rng(3).normal(0.0, 0.2, size=Mpnn.NPARAMS).astype(np.float32)
    th[-1] = np.log(np.e - 1.0)
    net = Mpnn(th)
    kw = dict(lam=20.0, r=1.0, n_inner=2, tol=1e-6, maxit=3000, persistent=False)
    S = Solver(U, np.concatenate([w.y0 for w in wls]), **kw)
    S.set_learned(net)
    ev, dg = (to_np(t) for t in S.get_factor())
    row0, edge0 = U.segments
    worst = 0.0
    for k, (w, p) in enumerate(zip(wls, parts)):
        Ss = Solver(p, w.y0, **kw)
        Ss.set_learned(net)
        es, ds = (to_np(t) for t in Ss.get_factor())
        worst = max(worst, np.abs(ev[edge0[k]:edge0[k + 1]] - es).max() / np.abs(es).max(),
                    np.abs(dg[row0[k]:row0[k + 1]] - ds).max() / np.abs(ds).max())
    print(f"factor batch vs solo max rel diff {worst:.2e}")
    assert worst <= 1e-6
    rhs = np.random.default_rng(4).normal(size=(U.n, wls[0].d))
    x, it, info = S.pcg(rhs, np.zeros_like(rhs))
    q = to_np(S.apply_A(x))
    for k in range(len(wls)):
        sl = slice(row0[k], row0[k + 1])
        res = np.linalg.norm(q[sl] - rhs[sl], axis=0) / np.linalg.norm(rhs[sl], axis=0)
        assert res.max() <= 1e-5, res.max()
    print(f"learned PCG on the batch: iterations {it}, rel res {info['rel_res_max']:.2e}")


@pytest.mark.parametrize("shape", ["persistent", "strips2"])
def test_batch64_full_size_sampled(shape):
    """The 64-image batch (128..512 x 128..384 pixels, d = 10) at its real size
    in the benchmark's launch configurations (the persistent kernel, and one
    launch per phase on image strips sized for two waves, which the autotuner
    picks for this batch): one SOC iteration, checked on sampled images against
    their solo runs in the same shape and, for the smallest image, the oracle;
    Frobenius and element-wise errors."""
    from paper_1612_06496_amd import Solver
    banner(f"batch64 full size, {shape}")
    wls = synth.make_batch("voronoi_batch64_8nbr")
    parts, U = build(wls)
    sizes = np.array([w.n for w in wls])
    small, large = int(np.argmin(sizes)), int(np.argmax(sizes))
    lam, r = fixed_penalties([wls[small]])
    # the smallest image starts from the oracle's D-orthonormal embedding (in
    # float32), so its step is compared from the same state on both sides
    g = oracle_graph(wls[small])
    Y0 = [w.y0 for w in wls]
    Y0[small] = O.orthonormalize_init(g, wls[small].y0).astype(np.float32)
    persistent = shape == "persistent"
    kw = dict(lam=lam, r=r, n_inner=wls[0].n_inner, tol=wls[0].tol, maxit=1000, persistent=persistent)

    def solver(graph, y0):
        Sx = Solver(graph, y0, **kw)
        if not persistent:
            Sx.set_launch_shape(persistent=False, strips=2)
        return Sx

    S = solver(U, np.concatenate(Y0))
    info = S.solve(1, info=True)
    if persistent:
        assert info["workgroups"] > 0
    else:
        assert info["workgroups"] == 0 and info["flags"] & 2
    row0, _ = U.segments
    Yg, Pg = to_np(S.get("Y")), to_np(S.get("P"))
    for k in (small, large, len(wls) // 2):
        Ss = solver(parts[k], Y0[k])
        Ss.solve(1)
        sl = slice(row0[k], row0[k + 1])
        Ys, Ps = to_np(Ss.get("Y")), to_np(Ss.get("P"))
        eY, eP = rel(Yg[sl], Ys), rel(Pg[sl], Ps)
        mY, mP = maxrel(Yg[sl], Ys), maxrel(Pg[sl], Ps)
        print(f"image {k} ({wls[k].H}x{wls[k].W}): batch vs solo Y {eY:.2e} ({mY:.2e} element-wise) "
              f"P {eP:.2e} ({mP:.2e})")
        assert eY <= 1e-5 and eP <= 1e-5
        assert mY <= 1e-4 and mP <= 1e-4
        Ss.close()
    Y = O.orthonormalize_init(g, Y0[small].astype(np.float64))
    solve = O.DirectSolver(O.system_matrix(g, lam, r))
    Y1, P1, _ = O.soc_outer_step(g, solve, Y, np.sqrt(g.D)[:, None] * Y, np.zeros_like(Y), lam, r,
                                 wls[small].n_inner)
    sl = slice(row0[small], row0[small + 1])
    eY, eP = rel(Yg[sl], Y1), rel(Pg[sl], P1)
    mY, mP = maxrel(Yg[sl], Y1), maxrel(Pg[sl], P1)
    print(f"smallest image vs oracle: Y {eY:.2e} ({mY:.2e} element-wise) P {eP:.2e} ({mP:.2e}); info {info}")
    assert eY <= 1e-5 and eP <= 1e-5
    assert mY <= 1e-4 and mP <= 1e-4
    S.close()


def test_autotune_restores_state_and_keeps_results():
    """The launch-shape autotuner restores the state it measured from, keeps
    one shape, and the tuned solver follows the default one (only the FP64
    summation order differs between shapes)."""
    from paper_1612_06496_amd import Solver
    banner("autotune")
    wls = synth.make_batch(BATCH)
    parts, U = build(wls)
    lam, r = fixed_penalties(wls)
    kw = dict(lam=lam, r=r, n_inner=wls[0].n_inner, tol=1e-6, maxit=3000)
    Y0 = np.concatenate([w.y0 for w in wls])
    S = Solver(U, Y0, **kw)
    before = [to_np(S.get(k)) for k in ("Y", "P", "B")]
    res = S.autotune(trials=1)
    print("autotune:", res)
    assert len(res) >= 2 and sum(x["chosen"] for x in res) == 1
    assert all(x["ms"] > 0 for x in res)
    after = [to_np(S.get(k)) for k in ("Y", "P", "B")]
    for b0, a0 in zip(before, after):
        assert np.array_equal(b0, a0)
    S.solve(2)
    R = Solver(U, Y0, **kw)
    R.solve(2)
    e = max(rel(to_np(S.get(k)), to_np(R.get(k))) for k in ("Y", "P"))
    print(f"tuned vs default rel err {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("shape", ["persistent", "strips", "rows"])
def test_several_dimensions_in_one_launch(shape):
    """A d-sweep in one launch: copies of one image in a block-diagonal union,
    copy s embedded in d_s dimensions (Y0 of the largest d with the columns
    beyond d_s set to zero).  Each copy must match the same image solved alone
    at its d_s (GPU, FP64) and the oracle at d_s; the padded columns stay
    exactly zero; monitors count only the active columns."""
    from paper_1612_06496_amd import Graph, Solver
    banner(f"several d in one launch, {shape}")
    wl = synth.make_workload("voronoi48x40_r2", 0)
    dims = [2, 5, 8]
    dmax = max(dims)
    g = oracle_graph(wl)
    lam, r = 40.0, 4.0
    parts = [gpu_graph(wl) for _ in dims]
    U = Graph.union(parts)
    Y0s = [synth.smooth_y0(wl.H, wl.W, dd, 100 + dd).astype(np.float64) for dd in dims]
    Y0 = np.zeros((U.n, dmax))
    row0, _ = U.segments
    for k, (dd, y) in enumerate(zip(dims, Y0s)):
        Y0[row0[k]:row0[k + 1], :dd] = y
    kw = dict(lam=lam, r=r, n_inner=3, tol=1e-12, maxit=3000, fp64=True, persistent=(shape == "persistent"))
    S = Solver(U, Y0, **kw)
    if shape != "persistent":
        S.set_launch_shape(persistent=False, strips=1 if shape == "strips" else 0)
    info = S.solve(2, info=True)
    if shape == "persistent":
        assert info["workgroups"] > 0
    Yg, Pg, Bg = (to_np(S.get(k)) for k in ("Y", "P", "B"))
    mon = S.monitor()
    print(f"monitors {mon}")
    assert mon["constraint"] <= 1e-9
    for k, dd in enumerate(dims):
        sl = slice(row0[k], row0[k + 1])
        assert np.all(Yg[sl, dd:] == 0.0) and np.all(Pg[sl, dd:] == 0.0) and np.all(Bg[sl, dd:] == 0.0)
        Ss = Solver(parts[k], Y0s[k], **{**kw, "persistent": False})
        Ss.solve(2)
        eS = max(rel(Yg[sl, :dd], to_np(Ss.get("Y"))), rel(Pg[sl, :dd], to_np(Ss.get("P"))))
        ref = O.pfe_run(g, Y0s[k], lam, r, 2, 3)
        eO = max(rel(Yg[sl, :dd], ref.Y), rel(Pg[sl, :dd], ref.P))
        print(f"d = {dd}: vs solo {eS:.2e}, vs oracle {eO:.2e}")
        assert eS <= 1e-9 and eO <= 1e-9
        Ss.close()
    S.close()


def test_zero_column_before_a_nonzero_one_is_rejected():
    from paper_1612_06496_amd import Solver
    from paper_1612_06496_amd import _lib as L
    banner("padded columns must trail")
    wl = synth.make_workload("voronoi48x40_r2", 0)
    Y0 = synth.smooth_y0(wl.H, wl.W, 4, 3).astype(np.float64)
    Y0[:, 1] = 0.0
    with pytest.raises(L.PFEError):
        Solver(gpu_graph(wl), Y0, lam=10.0, r=1.0, n_inner=2, fp64=True)
