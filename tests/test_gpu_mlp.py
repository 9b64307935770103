"""The warm-start network's HIP kernels (bfloat16 matrix cores and the FP32
reference mode) against the FP64 MLP oracle, and the gain of the learned warm
start over the solver without it."""
import numpy as np
import pytest

from synth import meshgen as mg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _setup(n, d_in, H, d_out, seed=0):
    from oracle import mlp
    p = mlp.init(d_in, H, d_out, seed)
    rng = np.random.default_rng(seed + 1)
    X = rng.standard_normal((n, d_in))
    T = rng.standard_normal((n, d_out))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    return p, X, T, dev(p), dev(X), dev(T)


@pytest.mark.parametrize("shape", [(8192, 32, 256, 6), (300, 32, 256, 6), (77, 5, 40, 3), (16, 16, 16, 16),
                                   (1000, 33, 70, 5)])
@pytest.mark.parametrize("mode,tol", [(0, 1e-5), (1, 2e-2)])
def test_mlp_forward_and_gradient(shape, mode, tol):
    """Forward pass, loss and every parameter's gradient against the FP64
    oracle: the production shape (8192 rows, 32 -> 256 -> 256 -> 6, whose
    weight gradients split the batch over 32 planes), shapes with ragged tiles
    in every dimension and leading dimensions that rule out 16-byte loads."""
    import paper_1511_04355_amd as afs
    from oracle import mlp
    n, d_in, H, d_out = shape
    assert afs._lib.mlp_n_params(d_in, H, d_out) == mlp.n_params(d_in, H, d_out)
    p, X, T, pd, Xd, Td = _setup(n, d_in, H, d_out)
    # the oracle runs on the same FP32-rounded inputs
    p32, X32 = p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64)
    Yo, _ = mlp.forward(p32, X32, d_in, H, d_out)
    Y = afs._lib.mlp_forward(pd, Xd, d_in, H, d_out, mode).cpu().numpy()
    assert np.max(np.abs(Y - Yo)) <= tol * np.max(np.abs(Yo))
    lo, go = mlp.loss_and_grad(p32, X32, T.astype(np.float32).astype(np.float64), d_in, H, d_out)
    loss, g = afs._lib.mlp_loss_grad(pd, Xd, Td, d_in, H, d_out, mode)
    g = g.cpu().numpy()
    assert abs(loss.item() - lo) <= tol * lo
    assert np.max(np.abs(g - go)) <= tol * np.max(np.abs(go))


def test_adam_step_matches_oracle():
    import paper_1511_04355_amd as afs
    from oracle import mlp
    rng = np.random.default_rng(2)
    p, g = rng.standard_normal(1000), rng.standard_normal(1000)
    m, v = 0.1 * rng.standard_normal(1000), np.abs(rng.standard_normal(1000))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    pd, gd, md, vd = dev(p), dev(g), dev(m), dev(v)
    afs._lib.mlp_adam(pd, gd, md, vd, 7, lr=1e-2)
    po, mo, vo = mlp.adam_step(p, g, m, v, 7, lr=1e-2)
    assert np.max(np.abs(pd.cpu().numpy() - po)) < 1e-6
    assert np.max(np.abs(md.cpu().numpy() - mo)) < 1e-6
    assert np.max(np.abs(vd.cpu().numpy() - vo)) < 1e-5


@pytest.mark.parametrize("shape", [(8192, 32, 256, 6), (77, 5, 40, 3)])
def test_fused_train_step_equals_gradient_then_adam(shape):
    """afsbem_mlp_train_step (gradient planes added and applied by Adam in one
    pass) against afsbem_mlp_loss_grad followed by afsbem_mlp_adam on a copy of
    the same state (both pinned to the oracle above): same loss, same
    parameters and moments after three steps."""
    import paper_1511_04355_amd as afs
    n, d_in, H, d_out = shape
    _, _, _, pd, Xd, Td = _setup(n, d_in, H, d_out, seed=7)
    p1, p2 = pd.clone(), pd.clone()
    m1, v1 = torch.zeros_like(pd), torch.zeros_like(pd)
    m2, v2 = torch.zeros_like(pd), torch.zeros_like(pd)
    for t in range(1, 4):
        l1 = afs._lib.mlp_train_step(p1, Xd, Td, m1, v1, t, d_in, H, d_out, lr=1e-3)
        l2, g = afs._lib.mlp_loss_grad(p2, Xd, Td, d_in, H, d_out, 1)
        afs._lib.mlp_adam(p2, g, m2, v2, t, lr=1e-3)
        assert abs(l1.item() - l2.item()) <= 1e-6 * abs(l2.item())
    for a, b in ((p1, p2), (m1, m2), (v1, v2)):
        assert torch.max(torch.abs(a - b)).item() <= 1e-6 * max(torch.max(torch.abs(b)).item(), 1e-30)


def test_training_reduces_loss():
    import paper_1511_04355_amd as afs
    n, d_in, H, d_out = 512, 8, 64, 6
    p, X, _, pd, Xd, _ = _setup(n, d_in, H, d_out, seed=4)
    T = np.sin(X[:, :d_out]) * np.cos(X[:, 1:2])
    Td = torch.from_numpy(T.astype(np.float32)).cuda()
    m, v = torch.zeros_like(pd), torch.zeros_like(pd)
    losses = []
    for t in range(1, 201):
        loss, g = afs._lib.mlp_loss_grad(pd, Xd, Td, d_in, H, d_out, 1)
        afs._lib.mlp_adam(pd, g, m, v, t, lr=3e-3)
        losses.append(loss.item())
    assert losses[-1] < 0.2 * losses[0]


def test_learned_warm_start_gain_and_parity():
    """Cavity (1280 triangles), 24 frequencies, mixed precision: the learned
    start reaches the oracle's solutions and needs fewer operator
    applications than starting from zero."""
    import paper_1511_04355_amd as afs
    from oracle import bem
    mesh = mg.cavity(3)
    s = mg.cavity_frequencies(24)
    bc = torch.from_numpy(np.stack([np.asarray(mesh.bc_shape, np.complex128) / sk for sk in s])).cuda()
    counts, sols, starts = {}, {}, {}
    for name, warm in [("none", afs.WARM_NONE), ("prev", afs.WARM_PREV), ("learned", afs.WARM_LEARNED)]:
        P = afs.Problem.from_mesh(mesh)
        out = P.solve(s, bc, afs.SolveOptions(tol=1e-6, precision=afs.PREC_MIXED, warm_start=warm))
        assert max(x["rel_res_fp64"] for x in out["stats"]) <= 1e-6
        counts[name] = sum(x["iters"] for x in out["stats"])
        starts[name] = ["%.1e/%d" % (x["rel_res_start"], x["used_net"]) for x in out["stats"]]
        sols[name] = out["a"].cpu().numpy()
        P.close()
    print("operator applications over 24 frequencies:", counts, flush=True)
    print("starting residuals:", starts, flush=True)
    assert counts["learned"] < counts["none"]
    # the gate stops querying a network that does not lower the starting residual
    assert counts["learned"] <= counts["prev"] + 12
    for k in (5, 17):
        A, b = bem.assemble(mesh, s[k])
        xo = bem.solve_dense(A, b)
        assert np.linalg.norm(sols["learned"][k] - xo) / np.linalg.norm(xo) <= 1e-5
