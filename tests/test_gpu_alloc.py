"""Device memory through a caller's allocator (pfe_set_allocator, here
PyTorch's caching allocator) and cold-started PCG solves (pfe_params.cold_start),
through the C ABI."""
import gc

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, gpu_graph, mid_run_state, oracle_graph, penalties, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def run(wl, lam, r):
    from paper_1612_06496_amd import Solver
    G = gpu_graph(wl)
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=wl.n_inner, tol=1e-6, maxit=1000)
    S.solve(2)
    out = {k: to_np(S.get(k)) for k in ("Y", "P", "B")}
    return G, S, out


def test_torch_caching_allocator_owns_library_memory():
    from paper_1612_06496_amd import live_allocations, use_torch_allocator
    from paper_1612_06496_amd._lib import PFEError
    gc.collect()
    torch.cuda.synchronize()
    if live_allocations() != 0:
        pytest.skip("library objects of earlier tests are still alive")
    banner("library memory through the torch caching allocator")
    wl = synth.make_workload("voronoi96x80_8nbr", 0)
    g = oracle_graph(wl)
    lam, r = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    G0, S0, ref = run(wl, lam, r)
    with pytest.raises(PFEError):          # library memory is out: no switch
        use_torch_allocator(True)
    S0.close()
    G0.close()
    del S0, G0
    gc.collect()
    assert live_allocations() == 0
    base = torch.cuda.memory_allocated()
    use_torch_allocator(True)
    try:
        G, S, got = run(wl, lam, r)
        held = torch.cuda.memory_allocated() - base
        n_live = live_allocations()
        print(f"torch-accounted library memory {held / 1e6:.1f} MB in {n_live} allocations")
        assert n_live > 0 and held >= 3 * wl.n * wl.d * 4
        for k in ("Y", "P", "B"):
            assert np.array_equal(got[k], ref[k])
        S.close()
        G.close()
        del S, G
        gc.collect()
        assert live_allocations() == 0
        assert torch.cuda.memory_allocated() == base
    finally:
        gc.collect()
        if live_allocations() == 0:
            use_torch_allocator(False)


def test_cold_start_matches_oracle_and_runs_per_phase():
    """PCG from zero instead of the current Y: the SOC iteration still equals
    the oracle's (whose direct solves do not depend on a start), more CG
    iterations are needed, and the persistent shape is not used."""
    from paper_1612_06496_amd import Solver
    wl = synth.make_workload("voronoi96x80_8nbr", 0)
    banner("cold-started PCG")
    g = oracle_graph(wl)
    lam, r = penalties(wl, g, O.orthonormalize_init(g, wl.y0))
    solve, Y, P, B, _, _ = mid_run_state(g, wl, lam, r, 1, 0)
    Y1, P1, B1 = O.soc_outer_step(g, solve, Y, P, B, lam, r, wl.n_inner)
    iters = {}
    for warm in (True, False):
        S = Solver(gpu_graph(wl), Y, lam=lam, r=r, n_inner=wl.n_inner, tol=1e-12, maxit=3000, fp64=True,
                   init_ortho=False, persistent=True, warm_start=warm)
        S.set("Y", Y); S.set("P", P); S.set("B", B)
        info = S.step("outer", info=True)
        eY, eP = rel(to_np(S.get("Y")), Y1), rel(to_np(S.get("P")), P1)
        iters[warm] = info["cg_iters_total"]
        print(f"warm={warm}: Y {eY:.2e} P {eP:.2e}; CG iterations {info['cg_iters_total']}; "
              f"workgroups {info['workgroups']}")
        assert eY <= 1e-9 and eP <= 1e-9
        assert (info["workgroups"] > 0) == warm
    assert iters[False] > iters[True]
