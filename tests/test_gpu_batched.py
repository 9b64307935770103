"""GPU parity of the batched (lockstep) solve: many systems -- frequencies of
one mesh and meshes of uneven size -- in one call, each against the oracle's
LU solution of the same system.

Tolerances as for the single-system solves: FP64 relative L2 1e-6 with GMRES
tolerance 1e-9 (the operators here have condition numbers well below 1e3);
mixed precision relative L2 1e-5 with tolerance 1e-6.  The reported residual
must be the oracle operator's residual.
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


def _tetra():
    return mg.Mesh(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]),
                   np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32),
                   np.array([0, 0, 1, 0], np.int8),
                   np.array([[0, 0, 1.0], [0.3, 0, 0], [0, 0, 0], [1, 1, 1.0]]))


def _bcs(mesh, s):
    return np.stack([np.asarray(mesh.bc_shape, np.complex128) / sk for sk in s]) if len(s) else \
        np.zeros((0, mesh.n_tri, 3), np.complex128)


def _check(mesh, s, bc, out, tol, err):
    from oracle import bem
    a = out["a"].cpu().numpy()
    for k, sk in enumerate(s):
        A, b = bem.assemble(mesh, sk, bc[k])
        xo = bem.solve_dense(A, b)
        st = out["stats"][k]
        assert st["status"] == 0, st
        assert st["rel_res_fp64"] <= tol
        assert np.linalg.norm(b - A @ a[k]) / np.linalg.norm(b) <= 1.5 * tol
        assert np.linalg.norm(a[k] - xo) / np.linalg.norm(xo) <= err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_cavity_L2_16_frequencies(prec):
    """The small cavity workload (320 triangles, 16 frequencies) in one call."""
    import paper_1511_04355_amd as afs
    mesh = mg.cavity(2)
    s = mg.cavity_frequencies(16)
    bc = _bcs(mesh, s)
    P = afs.Problem.from_mesh(mesh)
    tol, err = (1e-9, 1e-6) if prec == "fp64" else (1e-6, 1e-5)
    opts = afs.SolveOptions(tol=tol, precision=afs.PREC_FP64 if prec == "fp64" else afs.PREC_MIXED)
    print(f"[batched] cavity L2 x16 {prec}", flush=True)
    outs, rc = afs.solve_batched([P], [s], [torch.from_numpy(bc).cuda()], opts)
    assert rc == 0
    _check(mesh, s, bc, outs[0], tol, err)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("cap", [0, 3])
def test_batched_uneven_meshes(prec, cap):
    """Meshes of 4, 80, 64 and 320 triangles, 0 to 3 frequencies each, solved
    together; cap 3 forces several waves."""
    import paper_1511_04355_amd as afs
    meshes = [_tetra(), mg.cavity(1), mg.rod(2.0, 1.0, 3, 6), mg.cavity(2), mg.cavity(1)]
    s_lists = [np.array([0.25 + 3.1j, 0.5 + 0.0j]), mg.cavity_frequencies(3), np.array([0.5 + 0.3j]),
               mg.cavity_frequencies(5)[2:], np.array([], np.complex128)]
    bcs = [_bcs(m, s) for m, s in zip(meshes, s_lists)]
    probs = [afs.Problem.from_mesh(m) for m in meshes]
    tol, err = (1e-9, 1e-6) if prec == "fp64" else (1e-6, 1e-5)
    opts = afs.SolveOptions(tol=tol, precision=afs.PREC_FP64 if prec == "fp64" else afs.PREC_MIXED, batch=cap)
    print(f"[batched] uneven {prec} cap={cap}", flush=True)
    outs, rc = afs.solve_batched(probs, s_lists, [torch.from_numpy(b).cuda() for b in bcs], opts, want_ut=True)
    assert rc == 0
    for m, s, bc, o in zip(meshes, s_lists, bcs, outs):
        assert o["a"].shape[0] == len(s)
        _check(m, s, bc, o, tol, err)


def test_batched_u_t_split_rod():
    """u and t outputs of a mixed-condition mesh from the batched call."""
    import paper_1511_04355_amd as afs
    from oracle import bem
    mesh = mg.rod(2.0, 1.0, 3, 6)
    mat = (1.0, 0.0, 1.0)
    s = np.array([0.5 + 0.3j, 0.3 + 1.2j, 1.0 + 0.0j])
    bc = _bcs(mesh, s)
    P = afs.Problem.from_mesh(mesh, material=mat)
    outs, rc = afs.solve_batched([P], [s], [torch.from_numpy(bc).cuda()], afs.SolveOptions(tol=1e-10),
                                 want_ut=True)
    assert rc == 0
    for k, sk in enumerate(s):
        _, uo, to = bem.solve(mesh, sk, bc[k], mat=mat)
        assert np.linalg.norm(outs[0]["u"][k].cpu().numpy() - uo) / np.linalg.norm(uo) < 1e-8
        assert np.linalg.norm(outs[0]["t"][k].cpu().numpy() - to) / np.linalg.norm(to) < 1e-8


def test_batched_rejects_warm_start_and_matrix_free():
    import paper_1511_04355_amd as afs
    mesh = mg.cavity(1)
    s = mg.cavity_frequencies(2)
    P = afs.Problem.from_mesh(mesh)
    bc = torch.from_numpy(_bcs(mesh, s)).cuda()
    for o in (afs.SolveOptions(warm_start=afs.WARM_PREV), afs.SolveOptions(matrix_free=1)):
        with pytest.raises(afs.AfsbemError):
            afs.solve_batched([P], [s], [bc], o)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_cluster_preconditioner(prec):
    """Cluster block-Jacobi inside the lockstep solve: a seeded porous block
    (2,820 unknowns) and the small cavity, several frequencies each, against
    the oracle; fewer products than the point blocks on the porous block."""
    import paper_1511_04355_amd as afs
    meshes = [mg.random_block(7), mg.cavity(1)]
    s_lists = [np.array([0.25 + 0.5j, 0.25 + 1.5j, 0.25 + 2.5j]), mg.cavity_frequencies(3)]
    bcs = [_bcs(m, s) for m, s in zip(meshes, s_lists)]
    probs = [afs.Problem.from_mesh(m) for m in meshes]
    tol, err = (1e-9, 1e-6) if prec == "fp64" else (1e-6, 1e-5)
    iters = {}
    for pc in (0, 1):
        opts = afs.SolveOptions(tol=tol, precision=afs.PREC_FP64 if prec == "fp64" else afs.PREC_MIXED, precond=pc)
        outs, rc = afs.solve_batched(probs, s_lists, [torch.from_numpy(b).cuda() for b in bcs], opts)
        assert rc == 0
        iters[pc] = sum(x["iters"] for x in outs[0]["stats"])
        if pc == 1:
            for m, s, bc, o in zip(meshes, s_lists, bcs, outs):
                _check(m, s, bc, o, tol, err)
    print(f"[batched] porous block products: point {iters[0]}, clusters {iters[1]}", flush=True)
    assert iters[1] < iters[0]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_graph_replay_matches_eager(prec):
    """The captured 4-step graphs are replayed many times per call (every
    cycle of every outer step, with eager kernels, copies and host waits in
    between); the results must equal the eagerly launched solve exactly
    (same kernels, fixed-order reductions), on two calls in a row."""
    import paper_1511_04355_amd as afs
    meshes = [mg.cavity(1), mg.rod(2.0, 1.0, 3, 6), mg.cavity(2)]
    s_lists = [mg.cavity_frequencies(4), np.array([0.5 + 0.3j, 0.3 + 1.2j]), mg.cavity_frequencies(3)]
    bcs = [torch.from_numpy(_bcs(m, s)).cuda() for m, s in zip(meshes, s_lists)]
    probs = [afs.Problem.from_mesh(m) for m in meshes]
    kw = dict(tol=1e-9 if prec == "fp64" else 1e-7, precision=afs.PREC_FP64 if prec == "fp64" else afs.PREC_MIXED,
              restart=10)
    eager, rc = afs.solve_batched(probs, s_lists, bcs, afs.SolveOptions(no_graph=1, **kw))
    assert rc == 0
    for rep in range(2):
        outs, rc = afs.solve_batched(probs, s_lists, bcs, afs.SolveOptions(**kw))
        assert rc == 0
        for o, e in zip(outs, eager):
            assert torch.equal(o["a"], e["a"]), f"replay {rep}"
            assert [x["iters"] for x in o["stats"]] == [x["iters"] for x in e["stats"]]
