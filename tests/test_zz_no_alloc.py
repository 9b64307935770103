"""The allocation-free product entry point (afsbem_matvec_device_noalloc)
against afsbem_matvec_device, through the C ABI: every format and precision,
two calls in a row, the second on a smaller system, each checked to the
FP64 and FP32 product bars of the parity tests (the two differ only in the
column split of the partial sums, hence in summation order)."""
import numpy as np
import pytest

from synth import meshgen as mg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _case(afs, level, s, fmt):
    mesh = mg.cavity(level)
    P = afs.Problem.from_mesh(mesh)
    bc = torch.from_numpy(np.asarray(mesh.bc_shape, np.complex128) / s).cuda()
    A, A_lo, _, _ = P.assemble(s, bc, fmt=fmt)
    rng = np.random.default_rng(level)
    x = torch.from_numpy(rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)).cuda()
    return P, A, A_lo, x


@pytest.mark.parametrize("fmt,prec", [("c128", 0), ("split", 0), ("split", 1)])
def test_noalloc_matvec_matches_allocating_entry(fmt, prec):
    import paper_1511_04355_amd as afs
    f = afs.FMT_C128 if fmt == "c128" else afs.FMT_SPLIT
    bar = 1e-13 if prec == 0 else 1e-6
    for level, s in ((3, 0.25 + 1.3j), (2, 0.25 + 0.4j)):  # larger system first, then a smaller one
        P, A, A_lo, x = _case(afs, level, s, f)
        ref = P.matvec(A, A_lo, x, fmt=f, precision=prec)
        y = torch.full((P.N,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
        P.matvec_noalloc(A, A_lo, x, y, fmt=f, precision=prec)
        torch.cuda.synchronize()
        err = (torch.linalg.norm(y - ref) / torch.linalg.norm(ref)).item()
        print(f"noalloc {fmt} precision={prec} N={P.N}: rel diff {err:.2e}", flush=True)
        assert np.isfinite(err) and err <= bar
        del A, A_lo
        P.close()


def test_noalloc_matvec_rejects_bad_arguments():
    import paper_1511_04355_amd as afs
    P, A, A_lo, x = _case(afs, 1, 0.25 + 0.1j, afs.FMT_C128)
    y = torch.empty_like(x)
    with pytest.raises(afs.AfsbemError):
        P.matvec_noalloc(A, None, x, y, fmt=afs.FMT_SPLIT, precision=0)   # SPLIT without its lo plane
    with pytest.raises(afs.AfsbemError):
        P.matvec_noalloc(A, None, x, y, fmt=afs.FMT_C128, precision=1)   # FP32 needs SPLIT
