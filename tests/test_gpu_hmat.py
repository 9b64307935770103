"""The hierarchical far field (low-rank cross-approximation blocks + dense
near blocks) as the inner operator of the mixed matrix-free solve.

It approximates the operator by construction, so the bar is a property: the
product against the oracle's dense product (or, beyond the oracle's reach, the
FP64 on-the-fly product) to the requested accuracy, limited by FP32 storage;
and solves with it reach the FP64 true residual of the exact operator and the
oracle's LU solution, since the outer residual never uses it.
"""
import numpy as np
import pytest

from synth import meshgen as mg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _x(N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(N) + 1j * rng.standard_normal(N)


@pytest.mark.parametrize("name", ["cavity_L3", "block_seed3"])
def test_hmat_product_against_oracle(name):
    import paper_1511_04355_amd as afs
    from oracle import bem
    mesh = mg.cavity(3) if name == "cavity_L3" else mg.random_block(3)
    s = 0.25 + 1.3j
    P = afs.Problem.from_mesh(mesh)
    x = _x(P.N, 4)
    print(f"[hmat] {name} N={P.N}", flush=True)
    A, _ = bem.assemble(mesh, s)
    yo = A @ x
    errs = {}
    for eps in (1e-3, 1e-6):
        y, info = P.hmat_matvec(s, torch.from_numpy(x).cuda(), eps=eps)
        assert info["converged"], info
        errs[eps] = np.linalg.norm(y.cpu().numpy() - yo) / np.linalg.norm(yo)
        print(f"[hmat] eps {eps}: rel err {errs[eps]:.2e}, {info}", flush=True)
    assert info["n_lowrank"] > 0 and info["max_rank"] >= 1
    assert errs[1e-6] < 2e-5          # FP32 storage of the blocks and factors
    assert errs[1e-3] < 2e-2
    assert errs[1e-6] < errs[1e-3]


def test_hmat_solve_reaches_the_exact_residual():
    """matrix_free = 2: inner products through the hierarchical operator,
    outer FP64 residuals on the fly; the solution is the oracle's."""
    import paper_1511_04355_amd as afs
    from oracle import bem
    mesh = mg.cavity(3)
    s = np.array([0.25 + 0.7j, 0.25 + 2.0j])
    bc = np.stack([np.asarray(mesh.bc_shape, np.complex128) / sk for sk in s])
    P = afs.Problem.from_mesh(mesh)
    tol = 1e-6
    out = P.solve(s, torch.from_numpy(bc).cuda(),
                  afs.SolveOptions(tol=tol, precision=afs.PREC_MIXED, matrix_free=2, hmat_eps=1e-5))
    a = out["a"].cpu().numpy()
    for k, sk in enumerate(s):
        st = out["stats"][k]
        assert st["status"] == 0 and st["rel_res_fp64"] <= tol, st
        A, b = bem.assemble(mesh, sk)
        xo = bem.solve_dense(A, b)
        assert np.linalg.norm(a[k] - xo) / np.linalg.norm(xo) <= 1e-5
        assert np.linalg.norm(b - A @ a[k]) / np.linalg.norm(b) <= 1.01 * tol


@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_recycled_refinement_steps(tol):
    """Refinement steps after the first search the first inner solve's
    Krylov subspace plus new Arnoldi vectors (no_recycle = 0) or a fresh
    Krylov space (no_recycle = 1).  Both reach the FP64 residual of the exact
    operator and the oracle's LU solution; a coarse low-rank accuracy (1e-4)
    forces several steps, and the kept subspace needs fewer inner products."""
    import paper_1511_04355_amd as afs
    from oracle import bem
    mesh = mg.random_block(3)
    s = np.array([0.25 + 0.7j, 0.25 + 2.0j])
    bc = np.stack([np.asarray(mesh.bc_shape, np.complex128) / sk for sk in s])
    P = afs.Problem.from_mesh(mesh)
    outs = {}
    for nr in (0, 1):
        print(f"[hmat] recycle tol={tol} no_recycle={nr}", flush=True)
        outs[nr] = P.solve(s, torch.from_numpy(bc).cuda(),
                           afs.SolveOptions(tol=tol, precision=afs.PREC_MIXED, matrix_free=2, hmat_eps=1e-4,
                                            precond=1, restart=400, max_iter=4000, batch=1, no_recycle=nr))
    bar = 1e-5 if tol >= 1e-6 else 1e-7
    for k, sk in enumerate(s):
        A, b = bem.assemble(mesh, sk)
        xo = bem.solve_dense(A, b)
        for nr in (0, 1):
            st = outs[nr]["stats"][k]
            a = outs[nr]["a"][k].cpu().numpy()
            assert st["status"] == 0 and st["rel_res_fp64"] <= tol, (nr, st)
            assert st["refine_steps"] >= 2, (nr, st)
            assert np.linalg.norm(b - A @ a) / np.linalg.norm(b) <= 1.01 * tol
            assert np.linalg.norm(a - xo) / np.linalg.norm(xo) <= bar
    # products of the FP32 operator: all products less one FP64 residual per step
    inner = {nr: sum(st["iters"] - st["refine_steps"] for st in outs[nr]["stats"]) for nr in (0, 1)}
    print(f"[hmat] inner products: kept subspace {inner[0]}, fresh {inner[1]}", flush=True)
    assert inner[0] < inner[1]


def test_pipelined_schedules_give_the_same_solutions():
    """Frequencies one at a time (batch 1), two in flight with the next build
    beside the whole Krylov phase (0) or starting with the first FP64
    residual (2): the same kernels on the same inputs, so the same solutions
    (to rounding), each meeting the exact operator's FP64 residual; one
    frequency against the oracle's LU solution."""
    import paper_1511_04355_amd as afs
    from oracle import bem
    mesh = mg.random_block(3)
    s = np.array([0.25 + 0.4j, 0.25 + 0.9j, 0.25 + 1.5j, 0.25 + 2.2j])
    bc = np.stack([np.asarray(mesh.bc_shape, np.complex128) / sk for sk in s])
    P = afs.Problem.from_mesh(mesh)
    tol = 1e-6
    sols = {}
    for batch in (1, 0, 2):
        print(f"[hmat] schedule batch={batch}", flush=True)
        out = P.solve(s, torch.from_numpy(bc).cuda(),
                      afs.SolveOptions(tol=tol, precision=afs.PREC_MIXED, matrix_free=2, hmat_eps=1e-4, precond=1,
                                       restart=400, max_iter=4000, warm_start=afs.WARM_PREV, batch=batch))
        for st in out["stats"]:
            assert st["status"] == 0 and st["rel_res_fp64"] <= tol, (batch, st)
        sols[batch] = out["a"].cpu().numpy()
    for batch in (0, 2):
        d = np.linalg.norm(sols[batch] - sols[1], axis=1) / np.linalg.norm(sols[1], axis=1)
        assert np.all(d <= 1e-10), (batch, d)
    A, b = bem.assemble(mesh, s[2])
    xo = bem.solve_dense(A, b)
    assert np.linalg.norm(sols[2][2] - xo) / np.linalg.norm(xo) <= 1e-5


def test_hmat_option_checks():
    import paper_1511_04355_amd as afs
    mesh = mg.cavity(1)
    P = afs.Problem.from_mesh(mesh)
    bc = torch.zeros((1, P.n_tri, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(afs.AfsbemError):
        P.solve([0.3 + 0.5j], bc, afs.SolveOptions(matrix_free=2, precision=afs.PREC_FP64))
    with pytest.raises(afs.AfsbemError):
        P.hmat_matvec(0.3 + 0.5j, torch.zeros(P.N, dtype=torch.complex128, device="cuda"), eps=0.0)


@pytest.mark.timeout(300)
def test_hmat_product_full_size_27_voids():
    """40,320 unknowns (the 27-void block): the hierarchical product against
    the FP64 on-the-fly product on a random vector at two accuracies."""
    import paper_1511_04355_amd as afs
    mesh = mg.lattice_block(3, 20, 2, 1000)
    P = afs.Problem.from_mesh(mesh)
    s = complex(3.0 * np.log(10.0) / 300.0, 1.1)
    x = torch.from_numpy(_x(P.N, 6)).cuda()
    y_ref, _ = P.matvec_free(s, x, precision=0)
    for eps, bar in ((1e-4, 1e-3), (1e-6, 2e-5)):
        y, info = P.hmat_matvec(s, x, eps=eps)
        err = (torch.linalg.norm(y - y_ref) / torch.linalg.norm(y_ref)).item()
        print(f"[hmat] 27 voids, eps {eps}: rel err {err:.2e}, {info}", flush=True)
        assert info["converged"]
        assert err < bar


def test_hmat_without_low_rank_blocks_is_the_exact_operator():
    """A mesh too small for any admissible block: every block is dense, the
    product is the operator itself (to FP32 storage)."""
    import paper_1511_04355_amd as afs
    from oracle import bem
    mesh = mg.cavity(1)
    P = afs.Problem.from_mesh(mesh)
    s = 0.25 + 0.9j
    x = _x(P.N, 9)
    y, info = P.hmat_matvec(s, torch.from_numpy(x).cuda(), eps=1e-6)
    assert info["n_lowrank"] == 0 and info["converged"]
    A, _ = bem.assemble(mesh, s)
    yo = A @ x
    assert np.linalg.norm(y.cpu().numpy() - yo) / np.linalg.norm(yo) < 1e-6
