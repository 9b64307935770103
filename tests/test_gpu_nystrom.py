"""GPU parity of the Nystrom discretisation (curved six-node triangles, the
paper's own, Section 2.1) through the C ABI against the FP64 oracle on the
same inputs.

Tolerances as for the flat elements: FP64 entries to 1e-11 of the matrix
scale (same quadrature, different rounding order and series/closed-form
switch), FP64 solves to relative L2 1e-6 of the oracle's LU solution, the
mixed path to 1e-5.  Boundary values come from the oracle's own node normals
and are handed to both sides.
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


def _dense(A, N):
    return A[:, :N].cpu().numpy().T


def _mixed_cavity(level):
    """Cavity with alternating boundary kinds (both column kinds and both
    right-hand-side terms)."""
    m = mg.cavity_quadratic(level)
    m.bc_kind = (np.arange(m.n_tri) % 2).astype(np.int8)
    return m


def _point_force_bc(m, s):
    """The exact exterior field of a point force inside the cavity: the
    prescribed values and the values the solve must return."""
    from oracle import bem
    from oracle import nystrom as ny
    x0 = np.array([0.1, -0.05, 0.08])
    y, n, _ = ny.nodes(m)
    ue = np.array([bem.kernel(s, x0, y[i], n[i])[0][2] for i in range(len(y))])
    te = np.array([bem.kernel(s, x0, y[i], n[i])[1][2] for i in range(len(y))])
    kind = np.repeat(m.bc_kind, 6)
    return np.where(kind[:, None] == 0, te, ue), np.where(kind[:, None] == 0, ue, te)


def test_points_match_oracle_nodes():
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    m = mg.cavity_quadratic(1)
    P = afs.Problem.from_mesh(m)
    assert P.n_tri == m.n_nodes and P.N == m.n_unknowns
    y, n, w, kind = P.points()
    yo, no, wo = ny.nodes(m)
    assert np.max(np.abs(y - yo)) < 1e-14 and np.max(np.abs(n - no)) < 1e-14
    assert np.max(np.abs(w - wo)) < 1e-15
    assert np.all(kind == 0)


@pytest.mark.parametrize("level,s", [(0, 0.25 + 0.0j), (1, 0.3 + 0.9j), (1, 0.25 + 3.1j)])
def test_assembly_fp64_matches_oracle(level, s):
    """Every entry of A and b and the block-Jacobi inverses, all rows (N = 360
    and 1,440: several 64-row tiles with a ragged tail), mixed kinds."""
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    m = _mixed_cavity(level)
    bc, _ = _point_force_bc(m, s)
    print(f"[nystrom] assembly q{level} s={s}", flush=True)
    P = afs.Problem.from_mesh(m)
    A, _, b, pc = P.assemble(s, torch.from_numpy(bc).cuda(), fmt=afs.FMT_C128, with_precond=True)
    torch.cuda.synchronize()
    Ag = _dense(A, P.N)
    Ao, bo = ny.assemble(m, s, bc)
    assert np.max(np.abs(Ag - Ao)) <= 1e-11 * np.max(np.abs(Ao))
    assert np.max(np.abs(b.cpu().numpy() - bo)) <= 1e-11 * np.max(np.abs(bo))
    D = np.stack([Ao[3 * i:3 * i + 3, 3 * i:3 * i + 3] for i in range(P.n_tri)])
    Dinv = np.linalg.inv(D)
    assert np.max(np.abs(pc.cpu().numpy() - Dinv)) <= 1e-10 * np.max(np.abs(Dinv))


def test_assembly_split_planes():
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    m = mg.cavity_quadratic(1)
    s = 0.25 + 1.0j
    bc = ny.pressure_bc(m, s)
    P = afs.Problem.from_mesh(m)
    hi, lo, b, _ = P.assemble(s, torch.from_numpy(bc).cuda(), fmt=afs.FMT_SPLIT)
    torch.cuda.synchronize()
    Ao, _ = ny.assemble(m, s, bc)
    H = _dense(hi, P.N).astype(np.complex128)
    L = _dense(lo, P.N).astype(np.complex128)
    scale = np.max(np.abs(Ao))
    assert np.max(np.abs(H - Ao)) <= 1e-7 * scale
    assert np.max(np.abs(H + L - Ao)) <= 1e-11 * scale


def test_static_rigid_body_row_sums_on_the_gpu_matrix():
    """s = 0, traction prescribed everywhere: A = H and every row block sums
    to I for the exterior cavity (a property, independent of the oracle)."""
    import paper_1511_04355_amd as afs
    m = mg.cavity_quadratic(2)
    P = afs.Problem.from_mesh(m)
    bc = torch.zeros((P.n_tri, 3), dtype=torch.complex128, device="cuda")
    A, _, _, _ = P.assemble(0.0 + 0.0j, bc, fmt=afs.FMT_C128)
    torch.cuda.synchronize()
    Ag = _dense(A, P.N)
    rs = Ag.reshape(P.n_tri, 3, P.n_tri, 3).sum(axis=2)
    assert np.max(np.abs(rs - np.eye(3)[None])) < 5e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_matches_oracle_and_closed_form(precision):
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    from tests import analytic
    m = mg.cavity_quadratic(2)
    s = np.array([0.25 + 1.0j, 0.25 + 2.2j])
    _, nrm, _ = ny.nodes(m)
    bc = np.stack([ny.pressure_bc(m, sk, nrm) for sk in s])
    P = afs.Problem.from_mesh(m)
    prec = afs.PREC_FP64 if precision == "fp64" else afs.PREC_MIXED
    tol = 1e-8 if precision == "fp64" else 1e-6
    out = P.solve(s, torch.from_numpy(bc).cuda(), afs.SolveOptions(tol=tol, precision=prec))
    a = out["a"].cpu().numpy()
    for k, sk in enumerate(s):
        print(f"[nystrom] {precision} solve k={k}", flush=True)
        A, b = ny.assemble(m, sk, bc[k])
        xo = np.linalg.solve(A, b)
        st = out["stats"][k]
        assert st["status"] == 0 and st["rel_res_fp64"] <= tol
        assert np.linalg.norm(a[k] - xo) / np.linalg.norm(xo) <= (1e-6 if precision == "fp64" else 1e-5)
        assert np.linalg.norm(b - A @ a[k]) / np.linalg.norm(b) <= 1.01 * tol
        ur = analytic.cavity_ur(sk)
        un = np.einsum("ij,ij->i", a[k].reshape(-1, 3), -nrm)
        assert np.max(np.abs(un - ur)) / abs(ur) < 5e-4
    # u, t split: traction prescribed, so u = a and t = the given values
    assert np.allclose(out["u"].cpu().numpy().reshape(len(s), -1), a)
    assert np.allclose(out["t"].cpu().numpy(), bc)


def test_solve_mixed_conditions_manufactured():
    """Point-force field on alternating kinds: the solve returns the other half."""
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    m = _mixed_cavity(1)
    s = 0.25 + 1.0j
    bc, want = _point_force_bc(m, s)
    P = afs.Problem.from_mesh(m)
    out = P.solve([s], torch.from_numpy(bc[None]).cuda(), afs.SolveOptions(tol=1e-8, precision=afs.PREC_FP64))
    a = out["a"][0].cpu().numpy().reshape(-1, 3)
    xo = ny.solve(m, s, bc).reshape(-1, 3)
    assert np.linalg.norm(a - xo) / np.linalg.norm(xo) <= 1e-6
    assert np.linalg.norm(a - want) / np.linalg.norm(want) < 5e-3


def test_matrix_free_is_rejected():
    import paper_1511_04355_amd as afs
    m = mg.cavity_quadratic(0)
    P = afs.Problem.from_mesh(m)
    bc = torch.zeros((1, P.n_tri, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(afs.AfsbemError) as ei:
        P.solve([0.3 + 0.5j], bc, afs.SolveOptions(matrix_free=1))
    assert "Nystrom" in str(ei.value)


@pytest.mark.timeout(300)
def test_full_size_level3_sampled_rows_and_residual():
    """Level 3 (1,280 elements, 7,680 points, 23,040 unknowns): sampled rows
    of the GPU's A and b against the oracle's rows, and the mixed solve's
    residual bound on those rows."""
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    m = mg.cavity_quadratic(3)
    s = 0.25 + 1.9j
    _, nrm, _ = ny.nodes(m)
    bc = ny.pressure_bc(m, s, nrm)
    P = afs.Problem.from_mesh(m)
    print(f"[nystrom] full size N = {P.N}", flush=True)
    bct = torch.from_numpy(bc).cuda()
    A, _, b, _ = P.assemble(s, bct, fmt=afs.FMT_C128)
    rows = np.sort(np.random.default_rng(3).choice(P.n_tri, 24, replace=False))
    Ao, bo = ny.assemble(m, s, bc, rows=rows)
    idx = torch.from_numpy((3 * rows[:, None] + np.arange(3)[None]).reshape(-1)).cuda()
    Ag = A[:, :P.N].T[idx].cpu().numpy()
    bg = b.cpu().numpy()
    assert np.max(np.abs(Ag - Ao)) <= 1e-11 * np.max(np.abs(Ao))
    assert np.max(np.abs(bg[idx.cpu().numpy()] - bo)) <= 1e-11 * np.max(np.abs(bo))
    del A
    tol = 1e-6
    out = P.solve([s], bct[None], afs.SolveOptions(tol=tol, precision=afs.PREC_MIXED), want_ut=False)
    st = out["stats"][0]
    assert st["status"] == 0 and st["rel_res_fp64"] <= tol
    x = out["a"][0].cpu().numpy()
    r = np.max(np.abs(bo - Ao @ x))
    assert r <= 1.01 * tol * np.linalg.norm(bg)
    print(f"[nystrom] level 3: {st['iters']} products, sampled-row residual {r / np.linalg.norm(bg):.2e}", flush=True)


def test_batched_solve_of_two_nystrom_problems():
    """Two six-node problems of different sizes and kinds through one
    lockstep batched call, each frequency against the oracle's LU solution."""
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    m0, m1 = _mixed_cavity(0), mg.cavity_quadratic(1)
    s0 = np.array([0.25 + 0.5j, 0.25 + 1.3j])
    s1 = np.array([0.3 + 0.2j, 0.3 + 2.0j, 0.3 + 1.0j])
    bc0 = np.stack([_point_force_bc(m0, sk)[0] for sk in s0])
    _, nrm1, _ = ny.nodes(m1)
    bc1 = np.stack([ny.pressure_bc(m1, sk, nrm1) for sk in s1])
    probs = [afs.Problem.from_mesh(m0), afs.Problem.from_mesh(m1)]
    outs, rc = afs.solve_batched(probs, [s0, s1], [torch.from_numpy(bc0).cuda(), torch.from_numpy(bc1).cuda()],
                                 afs.SolveOptions(tol=1e-8, precision=afs.PREC_FP64))
    assert rc == 0
    for m, s, bc, o in ((m0, s0, bc0, outs[0]), (m1, s1, bc1, outs[1])):
        for k, sk in enumerate(s):
            assert o["stats"][k]["status"] == 0 and o["stats"][k]["rel_res_fp64"] <= 1e-8
            xo = ny.solve(m, sk, bc[k])
            a = o["a"][k].cpu().numpy()
            assert np.linalg.norm(a - xo) / np.linalg.norm(xo) <= 1e-6


def test_afs_driver_on_a_nystrom_problem():
    """Adaptive frequency sampling driving the six-node solve: every sampled
    response equals the oracle's discrete solution at that frequency."""
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    m = mg.cavity_quadratic(1)
    P = afs.Problem.from_mesh(m)
    _, nrm, _, _ = P.points()
    shape = -nrm
    dofs = np.sort(np.random.default_rng(8).choice(P.N, 6, replace=False))
    out = P.afs(afs.afs_params(20.0, 0.25, 64), shape, dofs, 4, load_kind=0, opts=afs.SolveOptions(tol=1e-10))
    assert out["converged"] and out["Nc"] <= 33
    for k in range(0, out["Nc"], 9):
        sk = out["s"][k]
        x = ny.solve(m, sk, shape / sk)
        assert np.max(np.abs(out["F"][k] - x[dofs])) <= 1e-7 * np.max(np.abs(x[dofs]))


@pytest.mark.parametrize("n_el", [1, 2])
def test_assembly_tiny_meshes(n_el):
    """One element (only the self rule: no near pair, no far pair) and two
    (near pairs only), against the oracle on every entry."""
    import paper_1511_04355_amd as afs
    from oracle import nystrom as ny
    full = mg.cavity_quadratic(0)
    used = np.unique(full.tri6[:n_el])
    remap = -np.ones(full.xyz.shape[0], np.int64)
    remap[used] = np.arange(len(used))
    m = mg.QuadMesh(full.xyz[used], remap[full.tri6[:n_el]].astype(np.int32), np.zeros(n_el, np.int8),
                    np.ones(n_el))
    s = 0.3 + 0.7j
    bc = ny.pressure_bc(m, s)
    P = afs.Problem.from_mesh(m)
    info = P.info()
    assert info["n_tri"] == 6 * n_el
    if n_el == 1:
        assert info["n_near_pairs"] == 0
    A, _, b, _ = P.assemble(s, torch.from_numpy(bc).cuda(), fmt=afs.FMT_C128)
    torch.cuda.synchronize()
    Ao, bo = ny.assemble(m, s, bc)
    assert np.max(np.abs(_dense(A, P.N) - Ao)) <= 1e-11 * np.max(np.abs(Ao))
    assert np.max(np.abs(b.cpu().numpy() - bo)) <= 1e-11 * np.max(np.abs(bo))


def test_degenerate_element_is_rejected():
    import paper_1511_04355_amd as afs
    xyz = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0.5, 0, 0], [1.5, 0, 0], [1, 0, 0.0]])
    m = mg.QuadMesh(xyz, np.array([[0, 1, 2, 3, 4, 5]], np.int32), np.zeros(1, np.int8), np.ones(1))
    with pytest.raises(afs.AfsbemError) as ei:
        afs.Problem.from_mesh(m)
    assert "degenerate" in str(ei.value)
