"""GPU parity of the learned preconditioner (network forward on MFMA, loss
chain, hand-written backward, Adam, PCG with M^{-1} = G^T G) against the FP64
oracle in oracle/learned.py.  Bounds: bf16 products -> 1e-2 relative on the
factor and the gradient; identity network -> the Jacobi PCG iterates."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, rel
from oracle import learned as LN

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def setup(lam=20.0, r=1.0, H=40, W=48, seed=3, stencil=8, fp64=False):
    from paper_1612_06496_amd import Graph, Solver
    wl = synth.grid_workload("t", H, W, 6, 0.05, seed, stencil=stencil, d=4)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    G = Graph.grid(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    S = Solver(G, wl.y0, lam=lam, r=r, n_inner=2, tol=1e-6, maxit=5000, fp64=fp64, persistent=False)
    return wl, g, G, S, LN.ScaledSystem(g, lam, r)


def random_params(seed, scale=0.3):
    th = np.random.default_rng(seed).normal(0.0, scale, size=LN.NPARAM)
    th[LN.NPARAM - 1] = LN.SOFTPLUS_ONE
    return th.astype(np.float32).astype(np.float64)


def oracle_edge_factor(th, SS):
    gv, dg = LN.factor(th, SS, bf16=True)
    up = SS.si < SS.sj                   # one slot per undirected edge, lexicographic
    return gv.numpy()[up], dg.numpy()


@pytest.mark.parametrize("stencil", [8, -2])
def test_factor_matches_oracle(stencil):
    from paper_1612_06496_amd import Mpnn
    banner(f"learned factor stencil={stencil}")
    wl, g, G, S, SS = setup(stencil=stencil)
    th = random_params(1)
    net = Mpnn(th)
    S.set_learned(net)
    ev, dg = S.get_factor()
    ev_o, dg_o = oracle_edge_factor(th, SS)
    e1 = np.abs(ev.cpu().numpy() - ev_o).max() / np.abs(ev_o).max()
    e2 = np.abs(dg.cpu().numpy() - dg_o).max() / np.abs(dg_o).max()
    print(f"factor: edge max rel {e1:.2e}, diag max rel {e2:.2e}")
    assert e1 <= 1e-2 and e2 <= 1e-2


def test_identity_network_is_jacobi():
    from paper_1612_06496_amd import Mpnn
    banner("identity network == Jacobi")
    wl, g, G, S, SS = setup()
    net = Mpnn(None)
    S.set_learned(net)
    ev, dg = S.get_factor()
    assert np.all(ev.cpu().numpy() == 0.0) and np.all(dg.cpu().numpy() == 1.0)
    rhs = np.random.default_rng(2).normal(size=(g.n, 4))
    x_l, it_l, _ = S.pcg(rhs, np.zeros_like(rhs))
    S.set_preconditioner("jacobi")
    x_j, it_j, _ = S.pcg(rhs, np.zeros_like(rhs))
    _, it_o = LN.pcg_preconditioned(SS.A, rhs, np.zeros_like(rhs), lambda q: q / SS.dA[:, None], 1e-6, 5000)
    print("iterations learned(identity)", it_l, "jacobi", it_j, "oracle", it_o)
    assert np.all(np.abs(it_l - it_o) <= 1)
    assert rel(x_l.cpu().numpy(), x_j.cpu().numpy()) <= 1e-5


def test_learned_pcg_matches_oracle():
    from paper_1612_06496_amd import Mpnn
    banner("learned PCG vs oracle")
    wl, g, G, S, SS = setup()
    th = random_params(4, scale=0.2)
    net = Mpnn(th)
    S.set_learned(net)
    rhs = np.random.default_rng(5).normal(size=(g.n, 4))
    x, it, info = S.pcg(rhs, np.zeros_like(rhs))
    gv, dg = LN.factor(th, SS)
    x_o, it_o = LN.pcg_preconditioned(SS.A, rhs, np.zeros_like(rhs),
                                      lambda q: LN.apply_preconditioner(gv, dg, SS, q), 1e-6, 5000)
    exact = O.DirectSolver(SS.A)(rhs)
    e = rel(x.cpu().numpy(), exact)
    print(f"iterations gpu {it} oracle {it_o}; solution rel err {e:.2e}; rel res {info['rel_res_max']:.2e}")
    assert info["rel_res_max"] <= 1e-6
    assert e <= 1e-4
    assert np.all(np.abs(it - it_o) <= 2)


@pytest.mark.parametrize("cols", [6, 8])
def test_gradient_matches_oracle_autograd(cols):
    """The training gradient against the oracle's autograd, with a sample
    count that takes the factor gradient's scalar path (6) and its 16-byte path
    (8)."""
    from paper_1612_06496_amd import Mpnn
    banner(f"learned gradient vs oracle, {cols} sample columns")
    wl, g, G, S, SS = setup(H=24, W=28)
    th = random_params(6, scale=0.2)
    net = Mpnn(th)
    R = np.random.default_rng(7).normal(size=(g.n, cols))
    loss_gpu = net.train_step(S, R, lr=0.0)
    grad_gpu = net.grad.astype(np.float64)
    rho = R / np.sqrt(SS.dA)[:, None]
    rho /= np.linalg.norm(rho, axis=0)
    loss_o, grad_o = LN.loss_and_grad(th, SS, rho, bf16=True)
    eg = np.linalg.norm(grad_gpu - grad_o) / np.linalg.norm(grad_o)
    print(f"loss gpu {loss_gpu:.6e} oracle {loss_o:.6e}; gradient rel err {eg:.2e}")
    assert abs(loss_gpu - loss_o) <= 1e-3 * loss_o
    assert eg <= 1e-2
    # params untouched with lr = 0
    assert np.array_equal(net.params, th.astype(np.float32))


def test_adam_step_matches_oracle():
    from paper_1612_06496_amd import Mpnn
    banner("adam step")
    wl, g, G, S, SS = setup(H=20, W=24)
    th = random_params(8, scale=0.2)
    net = Mpnn(th)
    R = np.random.default_rng(9).normal(size=(g.n, 4))
    net.train_step(S, R, lr=1e-3)
    g_gpu = net.grad.astype(np.float64)
    th1, _, _ = LN.adam_step(th, g_gpu, np.zeros_like(th), np.zeros_like(th), 1, 1e-3)
    assert np.abs(net.params - th1).max() <= 1e-6


@pytest.mark.parametrize("ratio", [1.0, 100.0])
def test_training_on_gpu_gains_on_held_out_image(ratio):
    """Train on residuals of one image's system, evaluate on another image."""
    from paper_1612_06496_amd import Graph, Mpnn, Solver
    banner(f"learned training gain lambda/r={ratio}")
    lam, r = ratio, 1.0
    wl_a = synth.grid_workload("a", 48, 56, 6, 0.05, 31, stencil=8, d=8)
    wl_b = synth.grid_workload("b", 48, 56, 6, 0.05, 32, stencil=8, d=8)
    Ga = Graph.grid(wl_a.feat, wl_a.H, wl_a.W, 8, 0.1)
    Gb = Graph.grid(wl_b.feat, wl_b.H, wl_b.W, 8, 0.1)
    Sa = Solver(Ga, wl_a.y0, lam=lam, r=r, n_inner=2, tol=1e-6, maxit=5000, persistent=False)
    Sb = Solver(Gb, wl_b.y0, lam=lam, r=r, n_inner=2, tol=1e-6, maxit=5000, persistent=False)
    net = Mpnn(random_params(0, 0.1).astype(np.float32))
    rng = np.random.default_rng(1)
    losses = []
    for step in range(200):
        R = rng.normal(size=(Ga.n, 16)).astype(np.float32)
        losses.append(net.train_step(Sa, R, lr=3e-3))
    rhs = rng.normal(size=(Gb.n, 8))
    Sb.set_preconditioner("jacobi")
    _, it_j, _ = Sb.pcg(rhs, np.zeros_like(rhs))
    Sb.set_learned(net)
    x, it_l, info = Sb.pcg(rhs, np.zeros_like(rhs))
    print(f"loss {losses[0]:.4f} -> {np.mean(losses[-10:]):.4f}; held-out iterations jacobi {it_j.max()} "
          f"learned {it_l.max()}")
    assert np.mean(losses[-10:]) < 0.8 * losses[0]
    assert it_l.max() < it_j.max()
    assert info["rel_res_max"] <= 1e-6


def test_learned_pcg_graph_replay_is_bitwise_neutral():
    from paper_1612_06496_amd import Mpnn, Solver
    banner("graph replay (learned PCG)")
    wl = synth.grid_workload("t", 40, 48, 6, 0.05, 3, stencil=8, d=4)
    G = __import__("gpu_helpers").gpu_graph(wl)
    net = Mpnn(random_params(4, scale=0.2))
    rhs = np.random.default_rng(5).normal(size=(wl.n, 4))
    out = []
    for graphs in (True, False):
        S = Solver(G, wl.y0, lam=20.0, r=1.0, n_inner=2, tol=1e-6, maxit=5000, persistent=False, graphs=graphs)
        S.set_learned(net)
        res = [S.pcg(rhs, np.zeros_like(rhs)) for _ in range(3)]     # three solves, the graph reused
        out.append(res)
    for (xa, ia, _), (xb, ib, _) in zip(out[0], out[1]):
        assert np.array_equal(ia, ib)
        assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())


def test_learned_pcg_on_edge_list_graph_matches_oracle():
    """General (non-stencil) slot layout: lower/upper neighbours chosen by column."""
    from paper_1612_06496_amd import Graph, Mpnn, Solver
    banner("learned PCG on a k-NN graph")
    wl = synth.edges_workload("gmm", 700, 8, 4, 6, 2, d=3)
    g = O.build_edge_graph(wl.n, wl.src, wl.dst, wl.dist2, wl.sigma)
    G = Graph.edges(wl.n, wl.src, wl.dst, wl.dist2, wl.sigma)
    S = Solver(G, wl.y0, lam=20.0, r=1.0, n_inner=2, tol=1e-6, maxit=5000, persistent=False)
    SS = LN.ScaledSystem(g, 20.0, 1.0)
    th = random_params(9, scale=0.2)
    S.set_learned(Mpnn(th))
    rhs = np.random.default_rng(10).normal(size=(g.n, 3))
    x, it, info = S.pcg(rhs, np.zeros_like(rhs))
    gv, dg = LN.factor(th, SS)
    _, it_o = LN.pcg_preconditioned(SS.A, rhs, np.zeros_like(rhs),
                                    lambda q: LN.apply_preconditioner(gv, dg, SS, q), 1e-6, 5000)
    exact = O.DirectSolver(SS.A)(rhs)
    e = rel(x.cpu().numpy(), exact)
    print(f"iterations gpu {it} oracle {it_o}; solution rel err {e:.2e}")
    assert info["rel_res_max"] <= 1e-6 and e <= 1e-4
    assert np.all(np.abs(it - it_o) <= 2)


def test_network_file_round_trip(tmp_path):
    """A network written by Mpnn.save and read by Mpnn.load has the same
    parameters (bitwise) and gives the same factor on a system."""
    from paper_1612_06496_amd import Mpnn, Solver
    from gpu_helpers import gpu_graph
    banner("network file round trip")
    th = np.random.default_rng(4).normal(0.0, 0.3, size=Mpnn.NPARAMS).astype(np.float32)
    net = Mpnn(th)
    path = tmp_path / "net.bin"
    net.save(path)
    net2 = Mpnn.load(path)
    assert np.array_equal(net2.params, th)
    wl = synth.make_workload("voronoi48x40_r2", 0)
    S = Solver(gpu_graph(wl), wl.y0, lam=20.0, r=1.0, n_inner=2, persistent=False)
    S.set_learned(net)
    f1 = [t.cpu().numpy() for t in S.get_factor()]
    S.set_learned(net2)
    f2 = [t.cpu().numpy() for t in S.get_factor()]
    assert all(np.array_equal(a, b) for a, b in zip(f1, f2))
