"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/afsbem.h declares; validation errors come back as status
codes without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afsbem.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(afsbem_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["afsbem_mesh_create", "afsbem_problem_create", "afsbem_assemble_device", "afsbem_matvec_device",
              "afsbem_solve_device", "afsbem_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1511_04355_amd as afs
    L = afs.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_error_string():
    import paper_1511_04355_amd as afs
    assert afs.version() == (0, 1)
    assert isinstance(afs.lib().afsbem_last_error(), bytes)


def test_mesh_validation_errors():
    import paper_1511_04355_amd as afs
    L = afs.lib()
    xyz = np.zeros((3, 3))
    tri = np.array([[0, 1, 5]], np.int32)  # index out of range
    out = ctypes.c_void_p()
    rc = L.afsbem_mesh_create(xyz.ctypes.data, 3, tri.ctypes.data, 1, ctypes.byref(out))
    assert rc == afs._lib.EINVAL
    assert b"out of range" in L.afsbem_last_error()
    rc = L.afsbem_mesh_create(None, 3, tri.ctypes.data, 1, ctypes.byref(out))
    assert rc == afs._lib.EINVAL
    xyz[0, 0] = np.nan
    tri = np.array([[0, 1, 2]], np.int32)
    rc = L.afsbem_mesh_create(xyz.ctypes.data, 3, tri.ctypes.data, 1, ctypes.byref(out))
    assert rc == afs._lib.EINVAL


def test_product_package_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_1511_04355_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "bem_oracle" not in text, f


def test_quadratic_mesh_validation_errors():
    import paper_1511_04355_amd as afs
    L = afs.lib()
    xyz = np.zeros((6, 3))
    tri6 = np.array([[0, 1, 2, 3, 4, 9]], np.int32)
    out = ctypes.c_void_p()
    rc = L.afsbem_mesh_create_quadratic(xyz.ctypes.data, 6, tri6.ctypes.data, 1, ctypes.byref(out))
    assert rc == afs._lib.EINVAL
    assert b"out of range" in L.afsbem_last_error()
    rc = L.afsbem_mesh_create_quadratic(xyz.ctypes.data, 5, tri6.ctypes.data, 1, ctypes.byref(out))
    assert rc == afs._lib.EINVAL


@pytest.mark.parametrize("name", ["cavity_L4", "block_seed3", "block_27_voids"])
def test_hmat_partition_covers_every_pair_once(name):
    """The hierarchical operator's block partition, built on the host: the
    blocks cover all n^2 element pairs (the recursion splits without overlap,
    so a full count means each pair once), no near pair falls in a low-rank
    block, the leaves tile the elements, and larger meshes get low-rank blocks."""
    import paper_1511_04355_amd as afs
    from synth import meshgen as mg
    mesh = {"cavity_L4": lambda: mg.cavity(4), "block_seed3": lambda: mg.random_block(3),
            "block_27_voids": lambda: mg.lattice_block(3, 20, 2, 1000)}[name]()
    info = afs.hmat_partition_info(mesh)
    n = info["n"]
    assert n == mesh.n_tri
    assert info["pairs_covered"] == n * n
    assert info["near_pairs_in_lowrank"] == 0
    assert info["leaf_elements"] == n
    assert info["n_lowrank"] > 0 and info["n_dense"] > 0
    assert info["leaf_list_entries"] >= info["n_dense"] + info["n_lowrank"]


def _flat_counts(mesh, ratio=2.0, max_depth=8):
    """Near pairs and subdivision leaves from the stated rule, on the oracle's
    element geometry: near if |c_m - c_n| < ratio h_n (h: longest edge); a near
    element splits into 4 at the edge midpoints while the piece fails the same
    test, up to max_depth."""
    from oracle import bem
    cen, _, _, hmax = bem.geometry(mesh)
    V = mesh.xyz[mesh.tri]
    near = leaves = 0

    def count(p, x, depth):
        c = p.mean(0)
        h = max(np.linalg.norm(p[0] - p[1]), np.linalg.norm(p[1] - p[2]), np.linalg.norm(p[2] - p[0]))
        if np.linalg.norm(x - c) < ratio * h and depth < max_depth:
            m01, m12, m20 = 0.5 * (p[0] + p[1]), 0.5 * (p[1] + p[2]), 0.5 * (p[2] + p[0])
            return sum(count(np.array(q), x, depth + 1) for q in
                       ((p[0], m01, m20), (m01, p[1], m12), (m20, m12, p[2]), (m01, m12, m20)))
        return 1

    for m in range(len(cen)):
        d = np.linalg.norm(cen - cen[m], axis=1)
        for n in np.nonzero(d < ratio * hmax)[0]:
            if n != m:
                near += 1
                leaves += count(V[n], cen[m], 0)
    return near, leaves


def _six_node_counts(mesh, ratio=2.0, max_depth=8):
    """The same rule for the Nystrom points: near if |y_i - x_e(1/3,1/3)| < ratio
    h_e (longest corner chord), subdivision of the parameter triangle with each
    piece's image tested (centre and longest corner chord), on the oracle's map."""
    from oracle import nystrom as ny
    y, _, _ = ny.nodes(mesh)
    P = mesh.xyz[mesh.tri6]
    cen = np.array([ny.q6_map(P[e], [[1 / 3, 1 / 3]])[0][0] for e in range(mesh.n_tri)])
    h = np.array([max(np.linalg.norm(P[e][a] - P[e][(a + 1) % 3]) for a in range(3)) for e in range(mesh.n_tri)])
    near = leaves = 0

    def count(Pe, q, x, depth):
        img, _, _ = ny.q6_map(Pe, np.vstack([q, q.mean(0)]))
        hh = max(np.linalg.norm(img[a] - img[(a + 1) % 3]) for a in range(3))
        if np.linalg.norm(x - img[3]) < ratio * hh and depth < max_depth:
            m01, m12, m20 = 0.5 * (q[0] + q[1]), 0.5 * (q[1] + q[2]), 0.5 * (q[2] + q[0])
            return sum(count(Pe, np.array(c), x, depth + 1) for c in
                       ((q[0], m01, m20), (m01, q[1], m12), (m20, m12, q[2]), (m01, m12, m20)))
        return 1

    ref = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    for i in range(len(y)):
        d = np.linalg.norm(cen - y[i], axis=1)
        for e in np.nonzero(d < ratio * h)[0]:
            if e != i // 6:
                near += 1
                leaves += count(P[e], ref, y[i], 0)
    return near, leaves


def test_plans_take_the_stated_near_and_subdivision_decisions():
    """The library's host plans (flat and six-node) against counts taken from
    the stated rules on the oracle's geometry: near pairs and subdivision leaves
    agree exactly."""
    import paper_1511_04355_amd as afs
    from synth import meshgen as mg
    m = mg.cavity(2)
    info = afs.plan_info(m)
    assert info["points"] == m.n_tri
    assert (info["near_pairs"], info["leaves"]) == _flat_counts(m)
    q = mg.cavity_quadratic(0)
    info = afs.plan_info(q)
    assert info["points"] == q.n_nodes
    assert (info["near_pairs"], info["leaves"]) == _six_node_counts(q)
