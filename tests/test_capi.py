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
