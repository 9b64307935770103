"""Host-side checks that need no GPU: the seeded input generators and the
bench contract's refusal of several GPUs."""
import os
import subprocess
import sys

import numpy as np

from synth import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_block_frequencies_seeded_band():
    s = mg.block_frequencies(24)
    eta, dw = mg.fsm_parameters(300.0, 3.0, 512)
    assert s.shape == (24,)
    assert np.allclose(s.real, eta)
    assert s[0].imag == 0.0 and np.all(np.diff(s.imag) >= 0)
    assert s.imag.max() <= 256 * dw
    assert np.array_equal(s, mg.block_frequencies(24))  # seeded
    assert not np.array_equal(s, mg.block_frequencies(24, seed=1))


def test_workload_meshes_have_the_stated_sizes():
    assert mg.cavity(2).n_tri == 320 and mg.cavity(4).n_tri == 5120
    assert mg.lattice_block(3, 20, 2, 1000).n_tri == 13440
    assert mg.lattice_block(4, 39, 3, 2000, rmax=0.45).n_tri == 100172
    sizes = [3 * mg.random_block(seed).n_tri for seed in range(16)]
    assert min(sizes) >= 2000 * 0.85 and max(sizes) <= 20000 * 1.15
    # closed, consistently oriented surfaces: every edge shared by two triangles in opposite directions
    m = mg.random_block(3)
    e = np.concatenate([m.tri[:, [0, 1]], m.tri[:, [1, 2]], m.tri[:, [2, 0]]])
    fwd = {tuple(x) for x in e}
    assert all((b, a) in fwd for a, b in fwd)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_six_node_cavity_mesh():
    """The six-node sphere: counts, every node on the sphere, each mid-edge node
    shared by the two elements of its edge (a conforming mesh), and the corner
    triangles oriented like the flat cavity's."""
    for L in (0, 1, 2):
        m = mg.cavity_quadratic(L)
        assert m.n_tri == 20 * 4 ** L and m.n_nodes == 120 * 4 ** L and m.n_unknowns == 360 * 4 ** L
        assert np.allclose(np.linalg.norm(m.xyz, axis=1), 1.0, atol=1e-14)
        owners = {}
        for e, t in enumerate(m.tri6):
            for a, mid in ((0, 3), (1, 4), (2, 5)):
                key = tuple(sorted((t[a], t[(a + 1) % 3])))
                owners.setdefault(key, set()).add(int(t[mid]))
        assert all(len(v) == 1 for v in owners.values())          # one mid node per edge
        assert len(owners) == 30 * 4 ** L                          # every edge of the closed surface
        flat = mg.cavity(L)
        assert np.array_equal(m.tri6[:, :3], flat.tri)
